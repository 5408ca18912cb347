// Dense semantic compositing: Eq. 3 with every Gaussian carrying a full
// distribution over the C classes (the dense representation the sparse
// top-k one replaces; supplement S.2.2 compares the two).  Same tiles,
// staging, culling and blending rules as the top-k forward; the semantic
// update of a blend touches all C class sums instead of k.
#include "pipeline.h"
#include "render_common.h"

namespace sgr {

constexpr int kDenseBatch = 64;  // entries per staged batch: one culling ballot

struct DenseArgs {
    TileArgs t;
    const uint32_t* pair_lin;  // record of a visible pair -> view * n + Gaussian
    int64_t n;
    const float* dense;     // [n][C]
};

size_t dense_lds_bytes(int C) {
    return (size_t)acc_floats(C) * sizeof(float) + (size_t)kDenseBatch * (4 * sizeof(float4) + sizeof(uint32_t)) +
           (size_t)kDenseBatch * C * sizeof(float);
}

__global__ __launch_bounds__(kBlock) void render_fwd_dense_kernel(DenseArgs d) {
    extern __shared__ __align__(16) float smem[];
    const TileArgs& a = d.t;
    const int gt = tile_of_block(blockIdx.x, gridDim.x, a.linear_tiles);
    if (gt >= a.num_tiles) return;
    if (a.counters[kStatus] & SGR_ECAPACITY) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int C = a.C;
    float* acc = smem;  // [C][257], column = owning thread
    float4* s_r0 = (float4*)(smem + acc_floats(C));
    float4* s_r1 = s_r0 + kDenseBatch;
    float4* s_r2 = s_r1 + kDenseBatch;
    float4* s_col = s_r2 + kDenseBatch;
    uint32_t* s_gid = (uint32_t*)(s_col + kDenseBatch);
    float* s_sv = (float*)(s_gid + kDenseBatch);  // [kDenseBatch][C]

    const int v = view_of_tile(a.views, a.V, gt);
    const ViewDev& vw = a.views[v];
    const int local = gt - vw.tile_off;
    const int tx = local % vw.tiles_x, ty = local / vw.tiles_x;
    const int px = tx * kTile + tile_px(tid), py = ty * kTile + tile_py(tid);
    const bool inside = px < vw.width && py < vw.height;
    const uint2 rg = a.ranges[gt];
    const uint32_t start = rg.x, end = rg.y;
    const int wx0 = tx * kTile + (wv & 1) * 8, wy0 = ty * kTile + (wv >> 1) * 8;
    for (int i = tid; i < C * kAccStride; i += kBlock) acc[i] = 0.f;

    float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, dd = 0.f, ss = 0.f;
    int ncon = 0;
    uint32_t last = start;
    bool done = !inside;
    const float amin = a.alpha_min, amax = a.alpha_max, tmin = a.t_min;

    for (uint32_t b0 = start; b0 < end; b0 += kDenseBatch) {
        if (__builtin_amdgcn_readfirstlane(__syncthreads_count(done)) == kBlock) break;
        const int nb = (int)min((uint32_t)kDenseBatch, end - b0);
        if (tid < nb) {
            const uint32_t g = a.owner[a.svals[b0 + tid]];
            const Proj p = a.srec[g];
            s_r0[tid] = p.r0;
            s_r1[tid] = p.r1;
            s_r2[tid] = p.r2;
            s_col[tid] = a.scol[g];
            const uint32_t lin = d.pair_lin[g];
            s_gid[tid] = (uint32_t)(lin - (uint64_t)(lin / d.n) * d.n);
        }
        __syncthreads();
        for (int e = tid; e < nb * C; e += kBlock) {  // each Gaussian's C values, row by row
            const int j = e / C, c = e - j * C;
            s_sv[e] = d.dense[(int64_t)s_gid[j] * C + c];
        }
        __syncthreads();
        bool hit = false;
        if (lane < nb) {
            const float4 q2 = s_r2[lane];
            const uint32_t rx = __float_as_uint(q2.x), ry = __float_as_uint(q2.y);
            hit = (int)(rx & 0xffffu) <= wx0 + 7 && (int)(rx >> 16) >= wx0 && (int)(ry & 0xffffu) <= wy0 + 7 &&
                  (int)(ry >> 16) >= wy0;
        }
        uint64_t todo = __ballot(hit);
        if (!done) {
            while (todo) {
                const int j = __builtin_ctzll(todo);
                todo &= todo - 1;
                const float4 q0 = s_r0[j], q1 = s_r1[j], q2 = s_r2[j];
                const uint32_t rx = __float_as_uint(q2.x), ry = __float_as_uint(q2.y);
                if (px < (int)(rx & 0xffffu) || px > (int)(rx >> 16) || py < (int)(ry & 0xffffu) ||
                    py > (int)(ry >> 16))
                    continue;
                float G, dx, dy;
                const float alpha = eval_alpha(q0, q1, px, py, amax, &G, &dx, &dy);
                if (alpha < amin) continue;
                const float Tn = T * (1.f - alpha);
                if (Tn < tmin) {
                    done = true;
                    break;
                }
                const float w = alpha * T;
                const float4 col = s_col[j];
                cr = fmaf(col.x, w, cr);
                cg = fmaf(col.y, w, cg);
                cb = fmaf(col.z, w, cb);
                dd = fmaf(col.w, w, dd);
                ss += w;
                const float* sv = s_sv + j * C;
                int c = 0;
                for (; c + 4 <= C; c += 4) {  // four reads, then four updates
                    float cur[4];
#pragma unroll
                    for (int q = 0; q < 4; q++) cur[q] = acc[(c + q) * kAccStride + tid];
#pragma unroll
                    for (int q = 0; q < 4; q++) acc[(c + q) * kAccStride + tid] = fmaf(sv[c + q], w, cur[q]);
                }
                for (; c < C; c++) acc[c * kAccStride + tid] = fmaf(sv[c], w, acc[c * kAccStride + tid]);
                T = Tn;
                ncon++;
                last = b0 + j + 1;
            }
        }
    }
    if (inside) {
        const int64_t pix = (int64_t)py * vw.width + px;
        const MapPtrs& o = a.maps[v];
        if (o.rgb) { o.rgb[3 * pix] = cr; o.rgb[3 * pix + 1] = cg; o.rgb[3 * pix + 2] = cb; }
        if (o.depth) o.depth[pix] = dd;
        if (o.sil) o.sil[pix] = ss;
        if (o.t_final) o.t_final[pix] = T;
        if (o.n_contrib) o.n_contrib[pix] = ncon;
        a.pix_T[vw.pix_off + pix] = T;
        a.pix_last[vw.pix_off + pix] = last;
    }
    float* out = a.maps[v].sem;
    if (!out) return;
    __syncthreads();
    write_rows_from_lds(smem, out, vw, C, tx, ty);
}

sgr_status launch_forward_dense(const Plan& P, const float* dense, const sgr_maps* out, char* ws, hipStream_t st) {
    DenseArgs d;
    memset(&d, 0, sizeof(d));
    d.t = make_tile_args(P, ws);
    std::vector<MapPtrs> mp(P.V);
    for (int v = 0; v < P.V; v++)
        mp[v] = MapPtrs{out[v].rgb, out[v].depth, out[v].sil, out[v].sem, out[v].t_final, out[v].n_contrib};
    set_view_table(d.t.maps, mp, ws + P.map_table, st);
    d.pair_lin = (const uint32_t*)(ws + P.pair_lin);
    d.n = P.n;
    d.dense = dense;
    const size_t lds = dense_lds_bytes(P.C);
    if (lds > device_max_lds()) return SGR_EUNSUPPORTED;
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void*)render_fwd_dense_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    const unsigned grid = (unsigned)(div_up(P.num_tiles, 8) * 8);
    render_fwd_dense_kernel<<<grid, kBlock, lds, st>>>(d);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

}  // namespace sgr
