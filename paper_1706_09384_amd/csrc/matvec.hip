// H-matrix-vector product (Section 3.1): y = sum over leaf blocks of the
// dense tile times x_sigma, or U (V^* x_sigma) for low-rank blocks.
//
// Three passes, no atomics, every output row written exactly once:
//   gather   x (original order, one column) -> xc (column-cluster order)
//   project  t_b = V_b^* xc[sigma_b] for every low-rank block (one workgroup
//            per block, one wave per column of V, lanes stream the column)
//   accum    one workgroup per leaf row cluster L: the sum over the dense
//            tiles of L and over the rows of every low-rank U whose row
//            cluster contains L; lanes own rows, waves split the task list,
//            LDS combines the waves; the result is scattered to original
//            order (or subtracted from b for the FP64 residual).
// Column-major tiles and factors make every inner load a coalesced column
// segment.  S is the storage real type, A the accumulation real type.
#include "internal.hpp"

namespace hm {

constexpr int kWave = 64;

template <typename A>
__device__ inline A wave_sum(A v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <typename S, typename A>
__global__ void gather_kernel(const cplx<S> *__restrict__ x, int64_t ldx, int32_t col,
                              const int32_t *__restrict__ perm, int64_t npts,
                              cplx<A> *__restrict__ xc) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 3 * npts) return;
    const int64_t p = k / 3, a = k - 3 * p;
    xc[k] = cvt<A>(x[(3 * (int64_t)perm[p] + a) * ldx + col]);
}

template <typename S, typename A>
__global__ void __launch_bounds__(256) project_kernel(const LowRankBlk *__restrict__ blk,
                                                      const cplx<S> *__restrict__ fac,
                                                      const cplx<A> *__restrict__ xc,
                                                      cplx<A> *__restrict__ t) {
    const LowRankBlk b = blk[blockIdx.x];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nw = blockDim.x / kWave;
    const int64_t rows = 3 * (int64_t)b.n;
    const cplx<A> *xs = xc + 3 * (int64_t)b.cb;
    for (int l = wave; l < b.r; l += nw) {
        const cplx<S> *v = fac + b.voff + l * rows;
        A re = 0, im = 0;
        for (int64_t i = lane; i < rows; i += kWave) {
            const cplx<A> vv = cvt<A>(v[i]);
            const cplx<A> xv = xs[i];
            // conj(v) * x
            re += vv.re * xv.re + vv.im * xv.im;
            im += vv.re * xv.im - vv.im * xv.re;
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) t[b.toff + l] = {re, im};
    }
}

// OUT = 0: y (type S) = A x; OUT = 1: r (double) = b - A x.
template <typename S, typename A, int OUT>
__global__ void __launch_bounds__(256) accum_kernel(
    const LeafRow *__restrict__ leaves, const Task *__restrict__ tasks,
    const DenseBlk *__restrict__ dblk, const LowRankBlk *__restrict__ lblk,
    const cplx<S> *__restrict__ dense, const cplx<S> *__restrict__ fac,
    const cplx<A> *__restrict__ xc, const cplx<A> *__restrict__ t,
    const int32_t *__restrict__ perm, void *__restrict__ yout, int64_t ldy, int32_t col,
    const double *__restrict__ bvec) {
    constexpr int RPL = 4;  // rows per lane per chunk
    __shared__ cplx<A> red[4][kWave * RPL];
    const LeafRow L = leaves[blockIdx.x];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nw = blockDim.x / kWave;
    const int32_t rows = 3 * L.m;
    for (int32_t r0 = 0; r0 < rows; r0 += kWave * RPL) {
        cplx<A> acc[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) acc[k] = {A(0), A(0)};
        for (int32_t ti = L.tbeg + wave; ti < L.tend; ti += nw) {
            const Task tk = tasks[ti];
            if (tk.kind == 0) {
                const DenseBlk d = dblk[tk.idx];
                const int64_t ld = 3 * (int64_t)d.m;
                const cplx<S> *tile = dense + d.off + 3 * (int64_t)tk.rowoff;
                const cplx<A> *xs = xc + 3 * (int64_t)d.cb;
                const int32_t ncol = 3 * d.n;
                for (int32_t jj = 0; jj < ncol; ++jj) {
                    const cplx<A> xv = xs[jj];
                    const cplx<S> *c = tile + jj * ld;
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        const int32_t row = r0 + lane + k * kWave;
                        if (row < rows) fma_(acc[k], cvt<A>(c[row]), xv);
                    }
                }
            } else {
                const LowRankBlk b = lblk[tk.idx];
                const int64_t ld = 3 * (int64_t)b.m;
                const cplx<S> *u = fac + b.uoff + 3 * (int64_t)tk.rowoff;
                const cplx<A> *tv = t + b.toff;
                for (int32_t l = 0; l < b.r; ++l) {
                    const cplx<A> tl = tv[l];
                    const cplx<S> *c = u + l * ld;
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        const int32_t row = r0 + lane + k * kWave;
                        if (row < rows) fma_(acc[k], cvt<A>(c[row]), tl);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) red[wave][lane + k * kWave] = acc[k];
        __syncthreads();
        for (int32_t q = threadIdx.x; q < kWave * RPL; q += blockDim.x) {
            const int32_t row = r0 + q;
            if (row < rows) {
                cplx<A> s = red[0][q];
                for (int w = 1; w < nw; ++w) s = s + red[w][q];
                const int32_t p = row / 3, a = row - 3 * p;
                const int64_t g = (3 * (int64_t)perm[L.rb + p] + a) * ldy + col;
                if (OUT == 0) {
                    static_cast<cplx<S> *>(yout)[g] = cvt<S>(s);
                } else {
                    const cplx<double> bb = {bvec[2 * g], bvec[2 * g + 1]};
                    static_cast<cplx<double> *>(yout)[g] = bb - cvt<double>(s);
                }
            }
        }
        __syncthreads();
    }
}

template <typename S, typename A>
void launch_matvec_col(const hm_matrix *M, const void *x, int64_t ldx, int32_t col, void *y,
                       int64_t ldy, const double *b, hipStream_t st) {
    const int64_t ny = M->ny;
    auto *xc = M->ws_xc.as<cplx<A>>();
    auto *tb = M->ws_t.as<cplx<A>>();
    const auto *perm_y = M->p.same ? M->perm_x.as<int32_t>() : M->perm_y.as<int32_t>();
    // The FP64 residual (b != nullptr) takes a complex128 x whatever the storage type.
    if (b == nullptr)
        hipLaunchKernelGGL((gather_kernel<S, A>), dim3(ceil_div(3 * ny, 256)), dim3(256), 0, st,
                           static_cast<const cplx<S> *>(x), ldx, col, perm_y, ny, xc);
    else
        hipLaunchKernelGGL((gather_kernel<double, A>), dim3(ceil_div(3 * ny, 256)), dim3(256), 0,
                           st, static_cast<const cplx<double> *>(x), ldx, col, perm_y, ny, xc);
    HM_HIP_CHECK(hipGetLastError());
    const auto *fac = M->lowrank.as<cplx<S>>();
    if (M->n_lblk > 0) {
        hipLaunchKernelGGL((project_kernel<S, A>), dim3(M->n_lblk), dim3(256), 0, st,
                           M->d_lblk.as<LowRankBlk>(), fac, xc, tb);
        HM_HIP_CHECK(hipGetLastError());
    }
    if (b == nullptr) {
        hipLaunchKernelGGL((accum_kernel<S, A, 0>), dim3(M->n_leaves), dim3(256), 0, st,
                           M->d_leaves.as<LeafRow>(), M->d_tasks.as<Task>(),
                           M->d_dblk.as<DenseBlk>(), M->d_lblk.as<LowRankBlk>(),
                           M->dense.as<cplx<S>>(), fac, xc, tb, M->perm_x.as<int32_t>(), y, ldy,
                           col, nullptr);
    } else {
        hipLaunchKernelGGL((accum_kernel<S, A, 1>), dim3(M->n_leaves), dim3(256), 0, st,
                           M->d_leaves.as<LeafRow>(), M->d_tasks.as<Task>(),
                           M->d_dblk.as<DenseBlk>(), M->d_lblk.as<LowRankBlk>(),
                           M->dense.as<cplx<S>>(), fac, xc, tb, M->perm_x.as<int32_t>(), y, ldy,
                           col, b);
    }
    HM_HIP_CHECK(hipGetLastError());
}

// Same three launches with HIP events between them; adds each kernel's
// duration (ms) to ms3[0..2] (gather, project, accum).
template <typename S>
void profile_matvec_col(const hm_matrix *M, const void *x, void *y, hipStream_t st, double *ms3) {
    using A = S;
    const int64_t ny = M->ny;
    auto *xc = M->ws_xc.as<cplx<A>>();
    auto *tb = M->ws_t.as<cplx<A>>();
    const auto *perm_y = M->p.same ? M->perm_x.as<int32_t>() : M->perm_y.as<int32_t>();
    hipEvent_t ev[4];
    for (auto &e : ev) HM_HIP_CHECK(hipEventCreate(&e));
    HM_HIP_CHECK(hipEventRecord(ev[0], st));
    hipLaunchKernelGGL((gather_kernel<S, A>), dim3(ceil_div(3 * ny, 256)), dim3(256), 0, st,
                       static_cast<const cplx<S> *>(x), 1, 0, perm_y, ny, xc);
    HM_HIP_CHECK(hipEventRecord(ev[1], st));
    const auto *fac = M->lowrank.as<cplx<S>>();
    if (M->n_lblk > 0)
        hipLaunchKernelGGL((project_kernel<S, A>), dim3(M->n_lblk), dim3(256), 0, st,
                           M->d_lblk.as<LowRankBlk>(), fac, xc, tb);
    HM_HIP_CHECK(hipEventRecord(ev[2], st));
    hipLaunchKernelGGL((accum_kernel<S, A, 0>), dim3(M->n_leaves), dim3(256), 0, st,
                       M->d_leaves.as<LeafRow>(), M->d_tasks.as<Task>(), M->d_dblk.as<DenseBlk>(),
                       M->d_lblk.as<LowRankBlk>(), M->dense.as<cplx<S>>(), fac, xc, tb,
                       M->perm_x.as<int32_t>(), y, 1, 0, nullptr);
    HM_HIP_CHECK(hipEventRecord(ev[3], st));
    HM_HIP_CHECK(hipEventSynchronize(ev[3]));
    for (int k = 0; k < 3; ++k) {
        float t = 0;
        HM_HIP_CHECK(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
        ms3[k] += t;
    }
    for (auto &e : ev) HM_HIP_CHECK(hipEventDestroy(e));
}

template void profile_matvec_col<float>(const hm_matrix *, const void *, void *, hipStream_t,
                                        double *);
template void profile_matvec_col<double>(const hm_matrix *, const void *, void *, hipStream_t,
                                         double *);

template void launch_matvec_col<float, float>(const hm_matrix *, const void *, int64_t, int32_t,
                                              void *, int64_t, const double *, hipStream_t);
template void launch_matvec_col<double, double>(const hm_matrix *, const void *, int64_t, int32_t,
                                                void *, int64_t, const double *, hipStream_t);
template void launch_matvec_col<float, double>(const hm_matrix *, const void *, int64_t, int32_t,
                                               void *, int64_t, const double *, hipStream_t);

}  // namespace hm
