// Sparse semantic state (Sec. 3.1, sparse semantic representation): the
// top-k classes a Gaussian keeps from the distribution it is initialised
// from, and updates of the kept values with the indices held fixed.
#include <cmath>

#include "pipeline.h"

namespace sgr {

// One thread per Gaussian.  The row is streamed once; (value, class) pairs
// are carried down a descending list of k in registers, where "better"
// means a larger value, or the same value and a smaller class.  NaN counts
// as -inf, so the list always fills with valid classes.
template <int KM>
__global__ __launch_bounds__(256) void topk_select_kernel(const float* __restrict__ dist,
                                                          const int64_t* __restrict__ pixel, int64_t n, int C, int k,
                                                          int renormalize, uint8_t* __restrict__ idx,
                                                          float* __restrict__ val) {
    const int64_t i = blockIdx.x * 256ll + threadIdx.x;
    if (i >= n) return;
    const float* row = dist + (pixel ? pixel[i] : i) * (int64_t)C;
    float bv[KM];
    int bi[KM];
#pragma unroll
    for (int m = 0; m < KM; m++) {
        bv[m] = -INFINITY;
        bi[m] = 0x7fffffff;
    }
    for (int c = 0; c < C; c++) {
        float cv = row[c];
        if (cv != cv) cv = -INFINITY;
        int ci = c;
#pragma unroll
        for (int m = 0; m < KM; m++) {
            if (m < k) {
                const bool better = cv > bv[m] || (cv == bv[m] && ci < bi[m]);
                const float tv = bv[m];
                const int ti = bi[m];
                bv[m] = better ? cv : tv;
                bi[m] = better ? ci : ti;
                cv = better ? tv : cv;
                ci = better ? ti : ci;
            }
        }
    }
    float s = 0.f;
#pragma unroll
    for (int m = 0; m < KM; m++) {
        if (m < k) {
            if (bv[m] == -INFINITY) bv[m] = 0.f;
            s += bv[m];
        }
    }
#pragma unroll
    for (int m = 0; m < KM; m++) {
        if (m < k) {
            idx[i * k + m] = (uint8_t)bi[m];
            val[i * k + m] = (renormalize && s > 0.f) ? bv[m] / s : bv[m];
        }
    }
}

__global__ __launch_bounds__(256) void topk_update_kernel(const float* __restrict__ dist,
                                                          const int64_t* __restrict__ pixel, int64_t n, int C, int k,
                                                          const uint8_t* __restrict__ idx, float rate,
                                                          float* __restrict__ val) {
    const int64_t e = blockIdx.x * 256ll + threadIdx.x;
    if (e >= n * k) return;
    const int64_t i = e / k;
    const int c = idx[e];
    const float obs = c < C ? dist[(pixel ? pixel[i] : i) * (int64_t)C + c] : 0.f;
    val[e] = (1.f - rate) * val[e] + rate * obs;
}

}  // namespace sgr

using namespace sgr;

extern "C" {

sgr_status sgr_topk_select(const float* dist, const int64_t* pixel, int64_t n, int32_t num_classes, int32_t k,
                           int32_t renormalize, uint8_t* sem_idx, float* sem_val, void* stream) {
    if (n < 0 || num_classes < 1 || num_classes > kMaxC || k < 1 || k > kMaxK || k > num_classes) return SGR_EINVAL;
    if (n == 0) return SGR_OK;
    if (!dist || !sem_idx || !sem_val) return SGR_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const unsigned grid = (unsigned)div_up(n, 256);
    if (k <= 4) topk_select_kernel<4><<<grid, 256, 0, st>>>(dist, pixel, n, num_classes, k, renormalize, sem_idx, sem_val);
    else if (k <= 8) topk_select_kernel<8><<<grid, 256, 0, st>>>(dist, pixel, n, num_classes, k, renormalize, sem_idx, sem_val);
    else if (k <= 16) topk_select_kernel<16><<<grid, 256, 0, st>>>(dist, pixel, n, num_classes, k, renormalize, sem_idx, sem_val);
    else topk_select_kernel<32><<<grid, 256, 0, st>>>(dist, pixel, n, num_classes, k, renormalize, sem_idx, sem_val);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

sgr_status sgr_topk_update(const float* dist, const int64_t* pixel, int64_t n, int32_t num_classes, int32_t k,
                           const uint8_t* sem_idx, float rate, float* sem_val, void* stream) {
    if (n < 0 || num_classes < 1 || num_classes > kMaxC || k < 1 || k > kMaxK || !(rate >= 0.f && rate <= 1.f))
        return SGR_EINVAL;
    if (n == 0) return SGR_OK;
    if (!dist || !sem_idx || !sem_val) return SGR_EINVAL;
    topk_update_kernel<<<(unsigned)div_up(n * k, 256), 256, 0, (hipStream_t)stream>>>(dist, pixel, n, num_classes, k,
                                                                                     sem_idx, rate, sem_val);
    return hipGetLastError() == hipSuccess ? SGR_OK : SGR_EHIP;
}

}  // extern "C"
