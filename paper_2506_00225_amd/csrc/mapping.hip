// Mapping-iteration helpers: the gradient of the per-keyframe mapping loss
// with respect to the rendered maps, and a fused Adam step with clamps.
#include "pipeline.h"

namespace sgr {

struct LossArgs {
    const float *rgb, *depth, *sil, *sem;   // rendered maps, [P][3], [P], [P], [P][C]
    const float *t_rgb, *t_depth;           // targets
    const int32_t* label;                   // [P]
    float *g_rgb, *g_depth, *g_sil, *g_sem; // outputs (g_sem dense [P][C])
    float* g_label;                         // [P] scratch: gradient of the label class
    int64_t P;
    int C;
    float w_depth, w_rgb, w_sil, w_ce, sil_thresh, inv_p;
};

// L = (1/P) sum_p [ m (w_d |D - D*| + w_c sum_ch |C - C*|) + w_s |S - 1| - w_ce ln max(P_label, 1e-6) ],
// m = [S > sil_thresh] (Sec. 3.1's silhouette-masked depth + 0.5 colour L1, plus silhouette and
// cross-entropy terms).  The mask is not differentiated.
__global__ __launch_bounds__(256) void loss_grad_pixels(LossArgs a) {
    const int64_t p = blockIdx.x * 256ll + threadIdx.x;
    if (p >= a.P) return;
    const float s = a.sil[p];
    const float m = s > a.sil_thresh ? a.inv_p : 0.f;
    const float dd = a.depth[p] - a.t_depth[p];
    a.g_depth[p] = m * a.w_depth * (dd > 0.f ? 1.f : (dd < 0.f ? -1.f : 0.f));
    for (int c = 0; c < 3; c++) {
        const float dc = a.rgb[3 * p + c] - a.t_rgb[3 * p + c];
        a.g_rgb[3 * p + c] = m * a.w_rgb * (dc > 0.f ? 1.f : (dc < 0.f ? -1.f : 0.f));
    }
    const float ds = s - 1.f;
    a.g_sil[p] = a.w_sil * a.inv_p * (ds > 0.f ? 1.f : (ds < 0.f ? -1.f : 0.f));
    const float pl = a.sem[p * a.C + a.label[p]];
    a.g_label[p] = pl > 1e-6f ? -a.w_ce * a.inv_p / pl : 0.f;
}

// Dense semantic gradient: zero except the label class of each pixel.
__global__ __launch_bounds__(256) void loss_grad_sem(const int32_t* __restrict__ label,
                                                     const float* __restrict__ g_label, int64_t total, int C,
                                                     float* __restrict__ g_sem) {
    const int64_t e4 = (blockIdx.x * 256ll + threadIdx.x) * 4;
    if (e4 >= total) return;
    float out[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int64_t e = e4 + q;
        out[q] = 0.f;
        if (e < total) {
            const int64_t p = e / C;
            const int c = (int)(e - p * C);
            if (c == label[p]) out[q] = g_label[p];
        }
    }
    if (e4 + 3 < total && ((((uintptr_t)(g_sem + e4)) & 15) == 0)) {
        *(float4*)(g_sem + e4) = make_float4(out[0], out[1], out[2], out[3]);
    } else {
        for (int q = 0; q < 4; q++)
            if (e4 + q < total) g_sem[e4 + q] = out[q];
    }
}

struct AdamSegs {
    sgr_adam_segment s[kMaxAdamSegs];
    int32_t count;
};

__global__ __launch_bounds__(256) void adam_kernel(AdamSegs segs, AdamParams h) {
    const sgr_adam_segment& sg = segs.s[blockIdx.y];
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < sg.n; i += (int64_t)gridDim.x * 256) {
        float m = sg.m[i], v = sg.v[i], p = sg.p[i];
        adam_update(sg.g[i], m, v, p, sg.lo, sg.hi, h);
        sg.m[i] = m;
        sg.v[i] = v;
        sg.p[i] = p;
    }
}

sgr_status launch_loss_grad(const LossArgs& a, hipStream_t st) {
    if (a.P == 0) return SGR_OK;
    loss_grad_pixels<<<(unsigned)div_up(a.P, 256), 256, 0, st>>>(a);
    const int64_t total = a.P * a.C;
    loss_grad_sem<<<(unsigned)div_up(div_up(total, 4), 256), 256, 0, st>>>(a.label, a.g_label, total, a.C, a.g_sem);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

sgr_status launch_adam(const sgr_adam_segment* segs, int n, float lr, float b1, float b2, float eps, int step,
                       hipStream_t st) {
    AdamSegs as;
    memset(&as, 0, sizeof(as));
    int64_t mx = 0;
    for (int i = 0; i < n; i++) {
        as.s[i] = segs[i];
        mx = std::max<int64_t>(mx, segs[i].n);
    }
    as.count = n;
    if (mx == 0) return SGR_OK;
    const AdamParams h = adam_params(lr, b1, b2, eps, step);
    const unsigned gx = (unsigned)std::min<int64_t>(div_up(mx, 256), 4096);
    adam_kernel<<<dim3(gx, (unsigned)n), 256, 0, st>>>(as, h);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

}  // namespace sgr

using namespace sgr;

extern "C" {

sgr_status sgr_mapping_loss_grad(const float* rgb, const float* depth, const float* sil, const float* sem,
                                 const float* t_rgb, const float* t_depth, const int32_t* label, int64_t num_pixels,
                                 int32_t num_classes, const float* weights, float* g_rgb, float* g_depth, float* g_sil,
                                 float* g_sem, float* scratch, void* stream) {
    if (num_pixels < 0 || num_classes < 1 || num_classes > kMaxC || !weights) return SGR_EINVAL;
    if (num_pixels > 0 && (!rgb || !depth || !sil || !sem || !t_rgb || !t_depth || !label || !g_rgb || !g_depth ||
                           !g_sil || !g_sem || !scratch))
        return SGR_EINVAL;
    LossArgs a;
    a.rgb = rgb; a.depth = depth; a.sil = sil; a.sem = sem;
    a.t_rgb = t_rgb; a.t_depth = t_depth; a.label = label;
    a.g_rgb = g_rgb; a.g_depth = g_depth; a.g_sil = g_sil; a.g_sem = g_sem; a.g_label = scratch;
    a.P = num_pixels;
    a.C = num_classes;
    a.w_depth = weights[0]; a.w_rgb = weights[1]; a.w_sil = weights[2]; a.w_ce = weights[3];
    a.sil_thresh = weights[4];
    a.inv_p = num_pixels > 0 ? 1.f / (float)num_pixels : 0.f;
    return launch_loss_grad(a, (hipStream_t)stream);
}

sgr_status sgr_adam_step(const sgr_adam_segment* segments, int32_t num_segments, float lr, float beta1, float beta2,
                         float eps, int32_t step, void* stream) {
    if (!segments || num_segments < 1 || num_segments > kMaxAdamSegs || step < 1 || !(lr >= 0.f) ||
        !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return SGR_EINVAL;
    for (int i = 0; i < num_segments; i++) {
        const sgr_adam_segment& s = segments[i];
        if (s.n < 0 || (s.n > 0 && (!s.p || !s.g || !s.m || !s.v)) || !(s.lo <= s.hi)) return SGR_EINVAL;
    }
    return launch_adam(segments, num_segments, lr, beta1, beta2, eps, step, (hipStream_t)stream);
}

}  // extern "C"
