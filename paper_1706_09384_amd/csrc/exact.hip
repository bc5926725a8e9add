// Sampled rows of the exact operator applied to a block of vectors: the
// reference against which an H-matrix product (Section 3.1) is measured, the
// same quantity as the row samples behind delta_H of Section 3.3.  Every
// entry block is evaluated again in FP64: the Green's tensor (eq. elasto_U /
// elasto_T, self blocks s I), or the collocation operator's element
// quadrature (Section 4).
//
// One workgroup per (sampled row, chunk of 4,096 columns): 256 column blocks
// at a time are evaluated into LDS (one per thread), then each thread
// accumulates its outputs (3 nrhs per row, strided over the threads) over the
// staged blocks.  Per-chunk partial sums are added in chunk order by a second
// kernel, so the result does not depend on scheduling.
#include "internal.hpp"

namespace hm {
namespace {

constexpr int kXrCols = 256;
constexpr int kXrChunk = 16 * kXrCols;
constexpr int kXrMaxRhs = 256;

template <bool Coll>
__global__ void __launch_bounds__(256)
    exact_rows_kernel(Geometry g, GreenParams<double> gp, const int32_t *__restrict__ rowpos,
                      const int32_t *__restrict__ perm_y, int64_t ny,
                      const cplx<double> *__restrict__ x, int32_t nrhs, double self_re,
                      double self_im, cplx<double> *__restrict__ part) {
    __shared__ cplx<double> Ks[kXrCols * 9];
    __shared__ int32_t col[kXrCols];
    const int tid = threadIdx.x;
    const int32_t pi = rowpos[blockIdx.x];
    const int64_t q0 = (int64_t)blockIdx.y * kXrChunk;
    const int64_t q1 = ny < q0 + kXrChunk ? ny : q0 + kXrChunk;
    const int nout = 3 * nrhs;
    cplx<double> acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int64_t base = q0; base < q1; base += kXrCols) {
        const int64_t q = base + tid;
        cplx<double> K[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) K[e] = {0, 0};
        if (q < q1) {
            const int32_t pj = (int32_t)q;
            if constexpr (Coll) {
                colloc_block<double>(g, gp, pi, pj, K);
            } else if (g.same && pi == pj) {
                K[0] = K[4] = K[8] = {self_re, self_im};
            } else {
                double nx = 0, nyy = 0, nz = 0;
                if (gp.kind == 1) {
                    nx = g.n[0][pj];
                    nyy = g.n[1][pj];
                    nz = g.n[2][pj];
                }
                green_block<double>(gp, g.x[0][pi] - g.y[0][pj], g.x[1][pi] - g.y[1][pj],
                                    g.x[2][pi] - g.y[2][pj], nx, nyy, nz, K);
            }
            col[tid] = perm_y[q];
        } else {
            col[tid] = 0;
        }
#pragma unroll
        for (int e = 0; e < 9; ++e) Ks[9 * tid + e] = K[e];
        __syncthreads();
        const int ncol = (int)(q1 - base < kXrCols ? q1 - base : kXrCols);
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int o = tid + 256 * u;
            if (o >= nout) break;
            const int a = o / nrhs, c = o - a * nrhs;
            cplx<double> s = acc[u];
            for (int jj = 0; jj < ncol; ++jj) {
                const cplx<double> *xj = x + 3 * (int64_t)col[jj] * nrhs + c;
                const cplx<double> *kr = Ks + 9 * jj + 3 * a;
                s = s + kr[0] * xj[0] + kr[1] * xj[nrhs] + kr[2] * xj[2 * (int64_t)nrhs];
            }
            acc[u] = s;
        }
        __syncthreads();
    }
    cplx<double> *out = part + ((int64_t)blockIdx.x * gridDim.y + blockIdx.y) * nout;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const int o = tid + 256 * u;
        if (o < nout) out[o] = acc[u];
    }
}

// y(3 r + a, c) = sum over chunks, in chunk order.
__global__ void exact_rows_sum_kernel(const cplx<double> *__restrict__ part, int32_t nrows,
                                      int32_t nch, int32_t nout, cplx<double> *__restrict__ y) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)nrows * nout) return;
    const int64_t r = k / nout, o = k - r * nout;
    cplx<double> s = {0, 0};
    for (int32_t ch = 0; ch < nch; ++ch) s = s + part[(r * nch + ch) * nout + o];
    y[r * nout + o] = s;
}

}  // namespace
}  // namespace hm

using namespace hm;

extern "C" hm_status hm_exact_rows(const hm_matrix *A, const int64_t *rows, int64_t nrows,
                                   const void *x, int32_t nrhs, void *y, void *stream) {
    HM_API_BEGIN
    if (A == nullptr || rows == nullptr || x == nullptr || y == nullptr)
        throw StatusError(HM_ERR_ARG, "NULL argument");
    if (A->plan_only) throw StatusError(HM_ERR_STATE, "matrix was built with plan_only");
    if (nrows < 1 || nrows > (1 << 20)) throw StatusError(HM_ERR_ARG, "nrows must lie in 1 .. 2^20");
    if (nrhs < 1 || nrhs > kXrMaxRhs) throw StatusError(HM_ERR_ARG, "nrhs must lie in 1 .. 256");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const ClusterTree &tx = A->rowtree();
    std::vector<int32_t> pos(A->nx);
    for (int64_t k = 0; k < A->nx; ++k) pos[tx.perm[k]] = (int32_t)k;
    std::vector<int32_t> rp(nrows);
    for (int64_t r = 0; r < nrows; ++r) {
        if (rows[r] < 0 || rows[r] >= A->nx) throw StatusError(HM_ERR_ARG, "row index out of range");
        rp[r] = pos[rows[r]];
    }
    const int64_t nch64 = ceil_div(A->ny, (int64_t)kXrChunk);
    const int32_t nch = (int32_t)nch64, nout = 3 * nrhs;
    DeviceBuf d_rows, part;
    d_rows.alloc(rp.size() * sizeof(int32_t));
    HM_HIP_CHECK(hipMemcpyAsync(d_rows.p, rp.data(), rp.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, st));
    part.alloc((size_t)nrows * nch * nout * sizeof(cplx<double>));
    const GreenParams<double> gp =
        make_green_params<double>(A->p.kernel, A->p.omega, A->p.lambda, A->p.mu, A->p.rho);
    const int32_t *perm_y = (A->p.same ? A->perm_x : A->perm_y).as<int32_t>();
    const auto kern = A->h_tri.empty() ? exact_rows_kernel<false> : exact_rows_kernel<true>;
    hipLaunchKernelGGL(kern, dim3((unsigned)nrows, (unsigned)nch), dim3(256), 0, st, A->geometry(), gp,
                       d_rows.as<int32_t>(), perm_y, A->ny, static_cast<const cplx<double> *>(x),
                       nrhs, A->p.self_re, A->p.self_im, part.as<cplx<double>>());
    const int64_t tot = nrows * (int64_t)nout;
    hipLaunchKernelGGL(exact_rows_sum_kernel, dim3((unsigned)ceil_div(tot, (int64_t)256)), dim3(256), 0,
                       st, part.as<cplx<double>>(), (int32_t)nrows, nch, nout,
                       static_cast<cplx<double> *>(y));
    HM_HIP_CHECK(hipGetLastError());
    // the row list and the partial sums are freed on return
    HM_HIP_CHECK(hipStreamSynchronize(st));
    return HM_OK;
    HM_API_END
}
