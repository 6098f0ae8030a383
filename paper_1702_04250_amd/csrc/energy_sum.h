// Final FP64 energy sums of a Poisson step, shared by the energy kernel of
// the rocFFT path and the last pass of the library's own transforms.
#pragma once

#include <hip/hip_runtime.h>

namespace pppm {

struct EnergySums {
    int ne;                  // k-space partial sums (blocks of the pass that took them)
    const double* epart;
    int nq;                  // particle-map partials: sum q, sum q^2, max |q| per block
    const double* qpart;
    double self_c;           // C g / sqrt(pi)
    double bg_c;             // C pi / (2 V g^2)
    double* eterms;          // [10] E, E_mesh, E_self, E_bg, Q, sum q^2, ...
    double* energy_out;      // caller's energy or null
};

// E_mesh from the k-space partials, Q and sum q^2 from the particle-map
// partials; E_self = -C g / sqrt(pi) sum q^2, E_bg = -C pi Q^2 / (2 V g^2).
// One block (any size up to 1024 threads, a multiple of 64) adds the
// partials in a fixed order, so the result does not depend on timing.  All
// threads of the block must call it.
__device__ __forceinline__ void energy_final_block(const EnergySums& es)
{
    __shared__ double red[3][16];
    double e = 0.0, qs = 0.0, q2 = 0.0;
    for (int i = threadIdx.x; i < es.ne; i += blockDim.x) e += es.epart[i];
    for (int i = threadIdx.x; i < es.nq; i += blockDim.x) {
        qs += es.qpart[3 * i];
        q2 += es.qpart[3 * i + 1];
    }
    for (int d = 32; d > 0; d >>= 1) {
        e += __shfl_down(e, d, 64);
        qs += __shfl_down(qs, d, 64);
        q2 += __shfl_down(q2, d, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wid] = e;
        red[1][wid] = qs;
        red[2][wid] = q2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double E = 0.0, Q = 0.0, Q2 = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            E += red[0][w];
            Q += red[1][w];
            Q2 += red[2][w];
        }
        const double e_self = -es.self_c * Q2;
        const double e_bg = -es.bg_c * Q * Q;
        const double total = E + e_self + e_bg;
        es.eterms[0] = total;
        es.eterms[1] = E;
        es.eterms[2] = e_self;
        es.eterms[3] = e_bg;
        es.eterms[4] = Q;
        es.eterms[5] = Q2;
        if (es.energy_out) *es.energy_out = total;
    }
}

}  // namespace pppm
