// Complex FP64 products on the matrix cores (v_mfma_f64_16x16x4f64), shared
// by the recompression and the randomized range finder.
#pragma once

#include "common.hpp"

namespace hm {

typedef double mf64x4 __attribute__((ext_vector_type(4)));

// C(i, j) = sum_k A(i, k) B(k, j) (complex FP64) on the matrix cores: one
// wave per 16 x 16 output tile, the workgroup's waves taking the tiles in
// turn; each 4-deep contraction step is three v_mfma_f64_16x16x4f64 (three
// real products per complex one).  Element accessors fa(i, k), fb(k, j), sink fc(i, j, v);
// the accessors are only called inside the bounds.  Ends with a barrier.
template <typename FA, typename FB, typename FC>
__device__ void mfma_gemm(int mC, int nC, int K, FA fa, FB fb, FC fc) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int tm = (mC + 15) >> 4, tn = (nC + 15) >> 4;
    const int g = lane >> 4;
    for (int t = wave; t < tm * tn; t += nw) {
        const int i0 = (t % tm) << 4, j0 = (t / tm) << 4;
        const int ia = i0 + (lane & 15), jb = j0 + (lane & 15);
        // three real products (Gauss): P1 = Re a Re b, P2 = Im a Im b,
        // P3 = (Re a + Im a)(Re b + Im b); Re = P1 - P2, Im = P3 - P1 - P2
        mf64x4 p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + g;
            const cplx<double> a = (ia < mC && k < K) ? fa(ia, k) : cplx<double>{0, 0};
            const cplx<double> b = (k < K && jb < nC) ? fb(k, jb) : cplx<double>{0, 0};
            p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.re, p1, 0, 0, 0);
            p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b.im, p2, 0, 0, 0);
            p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re + a.im, b.re + b.im, p3, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = i0 + 4 * e + g;
            if (i < mC && jb < nC) fc(i, jb, cplx<double>{p1[e] - p2[e], p3[e] - p1[e] - p2[e]});
        }
    }
    __syncthreads();
}

}  // namespace hm
