// Recompression of ACA factors (Section 3.2): B = U V^* = Q_U R_U R_V^* Q_V^*,
// truncated SVD of the small r x r core R_U R_V^* = P S L^*, then
// U' = Q_U P S^1/2 and V' = Q_V L S^1/2 keeping the leading singular values.
//
// GPU form (all FP64, whatever the storage precision):
//   gram     G_U = U^* U and G_V = V^* V, 32x32 output tiles per workgroup,
//            16-row slabs of both operands staged in LDS;
//   factor   per block, one workgroup: Cholesky G = R^* R (this is the R
//            factor of a thin QR of U, Q = U R^-1 never formed), core
//            M = R_U R_V^*, one-sided Jacobi SVD of M (parallel tournament
//            ordering, one wave per column pair), truncation by the
//            Frobenius tail, and the r x r' update matrices
//            W_U = R_V^* L_r S_r^-1/2,  W_V = R_U^* P_r S_r^-1/2,
//            which satisfy U W_U = Q_U P_r S_r^1/2 and V W_V = Q_V L_r S_r^1/2
//            without any triangular solve (R_U^-1 P = R_V^* L S^-1);
//   apply    U' = U W_U, V' = V W_V written to the compact final slab.
// A Cholesky pivot that is not positive (numerically dependent ACA columns)
// zeroes that row of R: the dependent column adds nothing to the range.
#include <climits>

#include "internal.hpp"

namespace hm {

// Per-block FP64 work area (complex doubles), 7 r x r column-major slots:
// 0 R_U (from G_U), 1 R_V (from G_V), 2 M (then M J), 3 J, 4 W_U, 5 W_V,
// 6 singular values and their ranking.
__host__ __device__ inline int64_t rc_slot(int32_t r, int s) { return (int64_t)s * r * r; }

struct GramItem {
    int32_t blk, which, ta, tc;   // which 0 = U, 1 = V; ta <= tc tile indices
};

constexpr int kGT = 32;   // output tile
constexpr int kGR = 16;   // rows per slab

template <typename R>
__global__ void __launch_bounds__(256) gram_kernel(const RcBlk *__restrict__ blks,
                                                   const GramItem *__restrict__ items,
                                                   const cplx<R> *__restrict__ fac,
                                                   cplx<double> *__restrict__ work) {
    __shared__ cplx<double> sa[kGR][kGT + 1];
    __shared__ cplx<double> sc[kGR][kGT + 1];
    const GramItem it = items[blockIdx.x];
    const RcBlk b = blks[it.blk];
    const int r = b.r;
    const int64_t rows = 3 * (int64_t)(it.which == 0 ? b.m : b.n);
    const cplx<R> *X = fac + (it.which == 0 ? b.uoff : b.voff);
    cplx<double> *G = work + b.goff + rc_slot(r, it.which);
    const int a0 = it.ta * kGT, c0 = it.tc * kGT;
    const int tid = threadIdx.x;
    // each thread owns 4 outputs: (a0 + ty*4 + k, c0 + tx) for k < 4
    const int tx = tid % kGT, ty = tid / kGT;   // ty in 0..7
    cplx<double> acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    for (int64_t i0 = 0; i0 < rows; i0 += kGR) {
        for (int q = tid; q < kGR * kGT; q += 256) {
            const int rr = q / kGT, cc = q % kGT;
            const int64_t row = i0 + rr;
            const int ca = a0 + cc, ccol = c0 + cc;
            sa[rr][cc] = (row < rows && ca < r) ? cvt<double>(X[(int64_t)ca * rows + row])
                                                : cplx<double>{0, 0};
            sc[rr][cc] = (row < rows && ccol < r) ? cvt<double>(X[(int64_t)ccol * rows + row])
                                                  : cplx<double>{0, 0};
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < kGR; ++rr) {
            const cplx<double> y = sc[rr][tx];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const cplx<double> x = sa[rr][ty * 4 + k];
                acc[k] = acc[k] + cmul(x, y);   // conj(x) * y
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int a = a0 + ty * 4 + k, c = c0 + tx;
        if (a < r && c < r && a <= c) {
            G[a + (int64_t)c * r] = acc[k];
            G[c + (int64_t)a * r] = conj(acc[k]);
        }
    }
}

// In-place upper Cholesky G = R^* R of an r x r Hermitian PSD matrix
// (column-major); entries below the diagonal are zeroed.
__device__ void chol_upper(cplx<double> *G, int r, double *sh_scalar) {
    const int tid = threadIdx.x;
    double dmax = 0;
    for (int k = 0; k < r; ++k) dmax = fmax(dmax, G[k + (int64_t)k * r].re);
    for (int k = 0; k < r; ++k) {
        if (tid == 0) {
            double d = G[k + (int64_t)k * r].re;
            for (int i = 0; i < k; ++i) d -= abs2(G[i + (int64_t)k * r]);
            const double rk = (d > 1e-15 * dmax && d > 0.0) ? sqrt(d) : 0.0;
            G[k + (int64_t)k * r] = {rk, 0.0};
            sh_scalar[0] = rk;
        }
        __syncthreads();
        const double rk = sh_scalar[0];
        for (int j = k + 1 + tid; j < r; j += blockDim.x) {
            cplx<double> s = G[k + (int64_t)j * r];
            for (int i = 0; i < k; ++i) s = s - cmul(G[i + (int64_t)k * r], G[i + (int64_t)j * r]);
            G[k + (int64_t)j * r] = rk > 0.0 ? (1.0 / rk) * s : cplx<double>{0, 0};
        }
        __syncthreads();
    }
    for (int64_t q = tid; q < (int64_t)r * r; q += blockDim.x) {
        const int i = (int)(q % r), j = (int)(q / r);
        if (i > j) G[q] = {0, 0};
    }
    __syncthreads();
}

__device__ inline double wave_sumd(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename R>
__global__ void __launch_bounds__(256) factor_kernel(const RcBlk *__restrict__ blks,
                                                     cplx<double> *__restrict__ work,
                                                     int32_t *__restrict__ newrank, double eps) {
    __shared__ double sh_s[1];
    __shared__ int sh_rot[4];
    __shared__ double sh_red[8];
    const RcBlk b = blks[blockIdx.x];
    const int r = b.r;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    if (r == 0) {
        if (tid == 0) newrank[blockIdx.x] = 0;
        return;
    }
    cplx<double> *W = work + b.goff;
    cplx<double> *RU = W + rc_slot(r, 0), *RV = W + rc_slot(r, 1), *M = W + rc_slot(r, 2),
                 *J = W + rc_slot(r, 3), *WU = W + rc_slot(r, 4), *WV = W + rc_slot(r, 5);
    chol_upper(RU, r, sh_s);
    chol_upper(RV, r, sh_s);
    // M = R_U R_V^*, J = I
    for (int64_t q = tid; q < (int64_t)r * r; q += 256) {
        const int i = (int)(q % r), j = (int)(q / r);
        cplx<double> s = {0, 0};
        for (int k = max(i, j); k < r; ++k)
            s = s + mulc(RU[i + (int64_t)k * r], RV[j + (int64_t)k * r]);
        M[q] = s;
        J[q] = (i == j) ? cplx<double>{1, 0} : cplx<double>{0, 0};
    }
    __syncthreads();
    // One-sided Jacobi with round-robin pairing over rr = r rounded up to even.
    const int rr = (r + 1) & ~1;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) sh_rot[0] = 0;
        __syncthreads();
        for (int round = 0; round < rr - 1; ++round) {
            for (int pr = wave; pr < rr / 2; pr += 4) {
                // tournament pairing: position 0 fixed, others rotate
                auto at = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (rr - 1); };
                int pcol = at(pr), qcol = at(rr - 1 - pr);
                if (pcol >= r || qcol >= r) continue;
                if (pcol > qcol) {
                    const int t = pcol;
                    pcol = qcol;
                    qcol = t;
                }
                cplx<double> *mp = M + (int64_t)pcol * r, *mq = M + (int64_t)qcol * r;
                double al = 0, be = 0, gr = 0, gi = 0;
                for (int i = lane; i < r; i += 64) {
                    const cplx<double> x = mp[i], y = mq[i];
                    al += abs2(x);
                    be += abs2(y);
                    gr += x.re * y.re + x.im * y.im;
                    gi += x.re * y.im - x.im * y.re;
                }
                al = wave_sumd(al);
                be = wave_sumd(be);
                gr = wave_sumd(gr);
                gi = wave_sumd(gi);
                const double ag = sqrt(gr * gr + gi * gi);
                if (ag == 0.0 || ag <= 1e-15 * sqrt(al * be)) continue;
                if (lane == 0) sh_rot[0] = 1;
                const double tau = (be - al) / (2.0 * ag);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                const cplx<double> ph = {gr / ag, -gi / ag};
                const cplx<double> v10 = (-s) * ph, v11 = c * ph;
                cplx<double> *jp = J + (int64_t)pcol * r, *jq = J + (int64_t)qcol * r;
                for (int i = lane; i < r; i += 64) {
                    const cplx<double> x = mp[i], y = mq[i];
                    mp[i] = c * x + y * v10;
                    mq[i] = s * x + y * v11;
                    const cplx<double> u = jp[i], w = jq[i];
                    jp[i] = c * u + w * v10;
                    jq[i] = s * u + w * v11;
                }
            }
            __syncthreads();
        }
        const int any = sh_rot[0];
        __syncthreads();
        if (!any) break;
    }
    // Singular values = column norms of M J, ranked in descending order.
    double *sv = reinterpret_cast<double *>(W + rc_slot(r, 6));   // r doubles
    int *idx = reinterpret_cast<int *>(sv + r);                   // r ints
    for (int c = wave; c < r; c += 4) {
        double s = 0;
        for (int i = lane; i < r; i += 64) s += abs2(M[i + (int64_t)c * r]);
        s = wave_sumd(s);
        if (lane == 0) sv[c] = sqrt(s);
    }
    __syncthreads();
    for (int c = tid; c < r; c += 256) {
        const double v = sv[c];
        int pos = 0;
        for (int k = 0; k < r; ++k) {
            const double w = sv[k];
            if (w > v || (w == v && k < c)) ++pos;
        }
        idx[pos] = c;
    }
    __syncthreads();
    if (tid == 0) {
        // keep = smallest k with sum_{i >= k} s_i^2 <= eps^2 sum s_i^2 (Frobenius tail)
        double tot = 0;
        for (int k = 0; k < r; ++k) tot += sv[idx[k]] * sv[idx[k]];
        int keep = 0;
        if (tot > 0.0) {
            double tail = 0;
            keep = r;
            for (int k = r; k >= 0; --k) {
                if (tail <= eps * eps * tot)
                    keep = k;
                else
                    break;
                if (k > 0) tail += sv[idx[k - 1]] * sv[idx[k - 1]];
            }
        }
        sh_rot[1] = keep;
    }
    __syncthreads();
    const int keep = sh_rot[1];
    // W_U[k][c] = sum_{j<=k} conj(R_V[j][k]) J[j][idx_c] / sqrt(s_c)
    // W_V[k][c] = sum_{i<=k} conj(R_U[i][k]) (M J)[i][idx_c] / s_c^(3/2)
    for (int64_t q = tid; q < (int64_t)r * keep; q += 256) {
        const int k = (int)(q % r), c = (int)(q / r);
        const int ic = idx[c];
        const double s = sv[ic];
        cplx<double> a = {0, 0}, bb = {0, 0};
        for (int j = 0; j <= k; ++j) a = a + cmul(RV[j + (int64_t)k * r], J[j + (int64_t)ic * r]);
        for (int i = 0; i <= k; ++i) bb = bb + cmul(RU[i + (int64_t)k * r], M[i + (int64_t)ic * r]);
        WU[q] = (1.0 / sqrt(s)) * a;
        WV[q] = (1.0 / (s * sqrt(s))) * bb;
    }
    if (tid == 0) newrank[blockIdx.x] = keep;
}

// U' = U W_U (3m x keep), V' = V W_V (3n x keep) into the compact slab.
template <typename R>
__global__ void __launch_bounds__(256) apply_kernel(const RcBlk *__restrict__ blks,
                                                    const cplx<R> *__restrict__ fac,
                                                    const cplx<double> *__restrict__ work,
                                                    const int32_t *__restrict__ newrank,
                                                    const int64_t *__restrict__ outu,
                                                    const int64_t *__restrict__ outv,
                                                    cplx<R> *__restrict__ out) {
    const int bi = blockIdx.y;
    const RcBlk b = blks[bi];
    const int r = b.r, keep = newrank[bi];
    if (keep == 0) return;
    const cplx<double> *W = work + b.goff;
    for (int which = 0; which < 2; ++which) {
        const int64_t rows = 3 * (int64_t)(which == 0 ? b.m : b.n);
        const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
        if (blockIdx.x * 256 >= rows) continue;
        const cplx<R> *X = fac + (which == 0 ? b.uoff : b.voff);
        const cplx<double> *T = W + rc_slot(r, which == 0 ? 4 : 5);
        cplx<R> *Y = out + (which == 0 ? outu[bi] : outv[bi]);
        if (row >= rows) continue;
        for (int c0 = 0; c0 < keep; c0 += 8) {
            cplx<double> acc[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] = {0, 0};
            for (int l = 0; l < r; ++l) {
                const cplx<double> x = cvt<double>(X[(int64_t)l * rows + row]);
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (c0 + k < keep) acc[k] = acc[k] + x * T[l + (int64_t)(c0 + k) * r];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (c0 + k < keep) Y[(int64_t)(c0 + k) * rows + row] = cvt<R>(acc[k]);
        }
    }
}

template <typename R>
void run_recompress(const std::vector<RcBlk> &blk, RcBlk *d_blk, const cplx<R> *acaslab,
                    double *work, int32_t *d_newrank, double eps, int32_t rmax, hipStream_t st) {
    if (blk.empty()) return;
    std::vector<GramItem> items;
    for (int32_t i = 0; i < (int32_t)blk.size(); ++i) {
        const int T = (int)ceil_div(blk[i].r, kGT);
        for (int w = 0; w < 2; ++w)
            for (int a = 0; a < T; ++a)
                for (int c = a; c < T; ++c) items.push_back({i, w, a, c});
    }
    (void)rmax;
    DeviceBuf d_items;
    if (!items.empty()) {
        d_items.alloc(items.size() * sizeof(GramItem));
        HM_HIP_CHECK(hipMemcpyAsync(d_items.p, items.data(), items.size() * sizeof(GramItem),
                                    hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(gram_kernel<R>, dim3((unsigned)items.size()), dim3(256), 0, st, d_blk,
                           d_items.as<GramItem>(), acaslab, reinterpret_cast<cplx<double> *>(work));
        HM_HIP_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(factor_kernel<R>, dim3((unsigned)blk.size()), dim3(256), 0, st, d_blk,
                       reinterpret_cast<cplx<double> *>(work), d_newrank, eps);
    HM_HIP_CHECK(hipGetLastError());
    // items (pageable) and d_items must outlive the copy and the kernels.
    HM_HIP_CHECK(hipStreamSynchronize(st));
}

template <typename R>
void run_recompress_apply(const std::vector<RcBlk> &blk, RcBlk *d_blk, const cplx<R> *acaslab,
                          const double *work, const int64_t *d_outu, const int64_t *d_outv,
                          const int32_t *d_newrank, cplx<R> *out, int32_t maxrows,
                          hipStream_t st) {
    if (blk.empty()) return;
    hipLaunchKernelGGL(apply_kernel<R>, dim3((unsigned)ceil_div(maxrows, 256), (unsigned)blk.size()),
                       dim3(256), 0, st, d_blk, acaslab,
                       reinterpret_cast<const cplx<double> *>(work), d_newrank, d_outu, d_outv,
                       out);
    HM_HIP_CHECK(hipGetLastError());
}

template void run_recompress<float>(const std::vector<RcBlk> &, RcBlk *, const cplx<float> *,
                                    double *, int32_t *, double, int32_t, hipStream_t);
template void run_recompress<double>(const std::vector<RcBlk> &, RcBlk *, const cplx<double> *,
                                     double *, int32_t *, double, int32_t, hipStream_t);
template void run_recompress_apply<float>(const std::vector<RcBlk> &, RcBlk *,
                                          const cplx<float> *, const double *, const int64_t *,
                                          const int64_t *, const int32_t *, cplx<float> *, int32_t,
                                          hipStream_t);
template void run_recompress_apply<double>(const std::vector<RcBlk> &, RcBlk *,
                                           const cplx<double> *, const double *, const int64_t *,
                                           const int64_t *, const int32_t *, cplx<double> *,
                                           int32_t, hipStream_t);

}  // namespace hm
