// Next-best-view selection (Sec. 3.2): candidate poses from the newly
// observed voxels of the exploration map, and the overall exploration
// criterion (Eq. 5-7) over the scored pool.
#include <cmath>

#include "pipeline.h"
#include "render_common.h"
#include "sort.h"

namespace sgr {

struct Lattice {
    int32_t nx, ny, nz;    // grid
    int32_t s;             // lattice spacing in voxels
    int32_t lx, ly, lz;    // lattice points per axis
    int32_t iz0;           // first layer
    float voxel, ox, oy, oz;
};

static bool make_lattice(const sgr_grid* g, const sgr_sampling* sm, Lattice* L) {
    if (!g || !sm || g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->voxel > 0.f) || !std::isfinite(g->voxel) ||
        !std::isfinite(g->origin[0]) || !std::isfinite(g->origin[1]) || !std::isfinite(g->origin[2]) ||
        !(sm->step > 0.f) || !std::isfinite(sm->step) || sm->directions < 1 || sm->directions > 4096 ||
        !std::isfinite(sm->z_min) || !std::isfinite(sm->z_max) || sm->z_max < sm->z_min)
        return false;
    if ((int64_t)g->nx * g->ny * g->nz >= ((int64_t)1 << 31)) return false;
    L->nx = g->nx; L->ny = g->ny; L->nz = g->nz;
    L->voxel = g->voxel; L->ox = g->origin[0]; L->oy = g->origin[1]; L->oz = g->origin[2];
    L->s = std::max(1, (int)std::lround(sm->step / g->voxel));
    // layers whose centre height lies in [z_min - voxel/2, z_max + voxel/2), same test as a reference in double
    int first = -1, last = -1;
    for (int iz = 0; iz < g->nz; iz++) {
        const double zc = (double)g->origin[2] + (iz + 0.5) * (double)g->voxel;
        if (zc >= (double)sm->z_min - 0.5 * g->voxel && zc < (double)sm->z_max + 0.5 * g->voxel) {
            if (first < 0) first = iz;
            last = iz;
        }
    }
    L->iz0 = first < 0 ? 0 : first;
    L->lz = first < 0 ? 0 : (last - first) / L->s + 1;
    L->lx = (g->nx + L->s - 1) / L->s;
    L->ly = (g->ny + L->s - 1) / L->s;
    return true;
}

static size_t lattice_points(const Lattice& L) { return (size_t)L.lx * L.ly * L.lz; }

struct CandWs {
    size_t flags, offs, partial, total, bytes;
};

static CandWs cand_layout(const Lattice& L) {
    CandWs w;
    const size_t n = std::max<size_t>(1, lattice_points(L));
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += (b + 255) & ~(size_t)255;
        return o;
    };
    w.flags = take(4 * n);
    w.offs = take(4 * n);
    w.partial = take(4 * scan_partial_words(n));
    w.total = take(4);
    w.bytes = off;
    return w;
}

__global__ __launch_bounds__(256) void site_flags_kernel(Lattice L, const uint8_t* __restrict__ now,
                                                         const uint8_t* __restrict__ before, uint32_t* flags) {
    const int64_t l = blockIdx.x * 256ll + threadIdx.x;
    const int64_t n = (int64_t)L.lx * L.ly * L.lz;
    if (l >= n) return;
    const int lx = (int)(l % L.lx), ly = (int)((l / L.lx) % L.ly), lz = (int)(l / ((int64_t)L.lx * L.ly));
    const int ix = lx * L.s, iy = ly * L.s, iz = L.iz0 + lz * L.s;
    const int64_t v = ((int64_t)iz * L.ny + iy) * L.nx + ix;
    flags[l] = (now[v] == 1 && !(before && before[v] == 1)) ? 1u : 0u;
}

// One thread per (lattice point, direction): the pose of a flagged site's
// direction j, computed in double precision and stored as float.
__global__ __launch_bounds__(256) void candidate_poses_kernel(Lattice L, int nd, const uint32_t* __restrict__ flags,
                                                              const uint32_t* __restrict__ offs, int64_t capacity,
                                                              float* __restrict__ poses, float* __restrict__ positions) {
    const int64_t t = blockIdx.x * 256ll + threadIdx.x;
    const int64_t n = (int64_t)L.lx * L.ly * L.lz;
    if (t >= n * nd) return;
    const int64_t l = t / nd;
    const int j = (int)(t - l * nd);
    if (!flags[l]) return;
    const int64_t v = (int64_t)offs[l] * nd + j;
    if (v >= capacity) return;
    const int lx = (int)(l % L.lx), ly = (int)((l / L.lx) % L.ly), lz = (int)(l / ((int64_t)L.lx * L.ly));
    const double p[3] = {(double)L.ox + (lx * L.s + 0.5) * (double)L.voxel,
                         (double)L.oy + (ly * L.s + 0.5) * (double)L.voxel,
                         (double)L.oz + (L.iz0 + lz * L.s + 0.5) * (double)L.voxel};
    // Fibonacci lattice direction j of nd
    const double z = 1.0 - (2.0 * j + 1.0) / nd;
    const double r = sqrt(fmax(0.0, 1.0 - z * z));
    const double phi = j * (M_PI * (3.0 - sqrt(5.0)));
    const double f[3] = {r * cos(phi), r * sin(phi), z};
    double u[3] = {0.0, 0.0, 1.0};
    if (fabs(f[2]) > 0.99) { u[0] = 1.0; u[2] = 0.0; }
    double rt[3] = {f[1] * u[2] - f[2] * u[1], f[2] * u[0] - f[0] * u[2], f[0] * u[1] - f[1] * u[0]};
    const double rn = sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
    for (int c = 0; c < 3; c++) rt[c] /= rn;
    const double d[3] = {f[1] * rt[2] - f[2] * rt[1], f[2] * rt[0] - f[0] * rt[2], f[0] * rt[1] - f[1] * rt[0]};
    const double* R[3] = {rt, d, f};
    float* o = poses + v * 12;
    for (int a = 0; a < 3; a++) {
        for (int c = 0; c < 3; c++) o[3 * a + c] = (float)R[a][c];
        o[9 + a] = (float)(-(R[a][0] * p[0] + R[a][1] * p[1] + R[a][2] * p[2]));
    }
    if (positions)
        for (int c = 0; c < 3; c++) positions[v * 3 + c] = (float)p[c];
}

__global__ void candidate_count_kernel(const uint32_t* total, int nd, int64_t* count) {
    *count = (int64_t)(*total) * nd;
}

// Eq. 5-7 in one workgroup, double precision, fixed reduction order.
__device__ __forceinline__ double block_sum(double x, double* red) {
    __syncthreads();
    red[threadIdx.x] = x;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    return red[0];
}

__device__ __forceinline__ double block_max(double x, double* red) {
    __syncthreads();
    red[threadIdx.x] = x;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    return red[0];
}

__global__ __launch_bounds__(256) void combine_kernel(int V, const uint32_t* __restrict__ n_empty,
                                                      const double* __restrict__ hsum, const float* __restrict__ pos,
                                                      float cx, float cy, float cz, double min_empty,
                                                      double* __restrict__ score, uint8_t* __restrict__ pruned,
                                                      int32_t* best) {
    __shared__ double red[256];
    __shared__ int32_t redi[256];
    const int tid = threadIdx.x;
    auto dist = [&](int v) {
        const double dx = (double)pos[3 * v] - cx, dy = (double)pos[3 * v + 1] - cy, dz = (double)pos[3 * v + 2] - cz;
        return sqrt(dx * dx + dy * dy + dz * dz);
    };
    double tn = 0.0, mh = -INFINITY, ml = -INFINITY;
    for (int v = tid; v < V; v += 256) {
        tn += (double)n_empty[v];
        mh = fmax(mh, hsum[v]);
        ml = fmax(ml, dist(v));
    }
    const double total = block_sum(tn, red);
    const double maxh = block_max(mh, red);
    const double maxl = block_max(ml, red);
    double sh = 0.0, sl = 0.0;
    for (int v = tid; v < V; v += 256) {
        sh += exp(hsum[v] - maxh);
        sl += exp(dist(v) - maxl);
    }
    const double Sh = block_sum(sh, red);
    const double Sl = block_sum(sl, red);
    double bs = -INFINITY;
    int32_t bi = -1;
    for (int v = tid; v < V; v += 256) {
        const double n = (double)n_empty[v];
        const double igeo = total > 0.0 ? n / total : 0.0;
        const double isem = exp(hsum[v] - maxh) / Sh;
        const double s = (1.0 - exp(dist(v) - maxl) / Sl) * igeo * isem;
        score[v] = s;
        const bool pr = n < min_empty;
        pruned[v] = pr ? 1 : 0;
        if (!pr && (bi < 0 || s > bs)) {  // strided order: the first index wins ties within a thread
            bs = s;
            bi = v;
        }
    }
    __syncthreads();
    red[tid] = bs;
    redi[tid] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            const double s2 = red[tid + o];
            const int32_t i2 = redi[tid + o];
            if (i2 >= 0 && (redi[tid] < 0 || s2 > red[tid] || (s2 == red[tid] && i2 < redi[tid]))) {
                red[tid] = s2;
                redi[tid] = i2;
            }
        }
        __syncthreads();
    }
    if (tid == 0) *best = redi[0];
}

}  // namespace sgr

using namespace sgr;

extern "C" {

size_t sgr_candidates_workspace_size(const sgr_grid* grid, const sgr_sampling* s) {
    Lattice L;
    if (!make_lattice(grid, s, &L)) return 0;
    return cand_layout(L).bytes;
}

sgr_status sgr_generate_candidates(const sgr_grid* grid, const uint8_t* free_now, const uint8_t* free_before,
                                   const sgr_sampling* s, int64_t capacity, float* poses, float* positions,
                                   int64_t* d_count, void* workspace, size_t workspace_bytes, void* stream) {
    Lattice L;
    if (!make_lattice(grid, s, &L)) return SGR_EINVAL;
    if (!free_now || !d_count || capacity < 0 || (capacity > 0 && !poses)) return SGR_EINVAL;
    const CandWs w = cand_layout(L);
    if (!workspace || workspace_bytes < w.bytes || ((uintptr_t)workspace & 255u)) return SGR_EINVAL;
    const size_t npts = lattice_points(L);
    if ((int64_t)npts * s->directions >= ((int64_t)1 << 31)) return SGR_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)workspace;
    uint32_t* flags = (uint32_t*)(ws + w.flags);
    uint32_t* offs = (uint32_t*)(ws + w.offs);
    uint32_t* total = (uint32_t*)(ws + w.total);
    zero_u32<<<1, 1, 0, st>>>(total);
    if (npts > 0) {
        site_flags_kernel<<<(unsigned)div_up((int64_t)npts, 256), 256, 0, st>>>(L, free_now, free_before, flags);
        scan_exclusive(flags, offs, host_count((uint32_t)npts), (uint32_t)npts, (uint32_t*)(ws + w.partial), total, 0,
                       nullptr, st);
        candidate_poses_kernel<<<(unsigned)div_up((int64_t)npts * s->directions, 256), 256, 0, st>>>(
            L, s->directions, flags, offs, capacity, poses, positions);
    }
    candidate_count_kernel<<<1, 1, 0, st>>>(total, s->directions, d_count);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

sgr_status sgr_combine_scores(int32_t num_views, const uint32_t* n_empty, const double* entropy_sum,
                              const float* positions, const float* current, int64_t pixels, float prune_fraction,
                              double* score, uint8_t* pruned, int32_t* best, void* stream) {
    if (num_views < 1 || !n_empty || !entropy_sum || !positions || !current || !score || !pruned || !best ||
        pixels < 1 || !(prune_fraction >= 0.f) || !std::isfinite(prune_fraction))
        return SGR_EINVAL;
    if (!std::isfinite(current[0]) || !std::isfinite(current[1]) || !std::isfinite(current[2])) return SGR_EINVAL;
    combine_kernel<<<1, 256, 0, (hipStream_t)stream>>>(num_views, n_empty, entropy_sum, positions, current[0],
                                                       current[1], current[2], (double)prune_fraction * (double)pixels,
                                                       score, pruned, best);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

}  // extern "C"
