// Restarted GMRES on the H-matrix (the iterative solver of Section 3.1).
//
// Reading (the paper names GMRES only): x0 = 0, no preconditioner,
// GMRES(restart) with classical Gram-Schmidt applied twice (CGS2) for the
// Arnoldi step, Givens rotations on the host for the small least-squares
// problem, convergence on the recursive residual, confirmed by an explicit
// residual at every restart.  The Gram-Schmidt coefficients and norms stay
// on the device; each Arnoldi step makes one device-to-host copy.  nrhs right-hand sides run as independent GMRES
// instances in lockstep: one multi-column H-matvec per iteration, the
// BLAS-1 kernels work on all columns at once, Hessenberg data per column.
// Complex64 operators: iterative refinement with an FP64 residual
// r = b - A_H x (FP64 arithmetic on the stored factors), an inner complex64
// GMRES on the normalised residual, and an FP64 update, until the FP64
// relative residual meets tol.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "internal.hpp"

extern "C" hm_status hm_matvec(const hm_matrix *A, const void *x, void *y, int32_t nrhs,
                               void *stream);
extern "C" hm_status hm_residual(const hm_matrix *A, const void *b, const void *x, void *r,
                                 int32_t nrhs, void *stream);

namespace hm {

using zd = std::complex<double>;

// partial[(blockIdx.x * nvec + i) * nrhs + c] = sum over this block's rows of conj(V_i) w
template <typename T>
__global__ void dots_kernel(const cplx<T> *__restrict__ V, int64_t vstride, int nvec,
                            const cplx<T> *__restrict__ w, int64_t len, int nrhs,
                            cplx<double> *__restrict__ partial) {
    __shared__ cplx<double> red[256];
    const int i = blockIdx.y;
    const cplx<T> *v = V + i * vstride;
    cplx<double> acc = {0, 0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += stride)
        acc = acc + cmul(cvt<double>(v[k]), cvt<double>(w[k]));
    red[threadIdx.x] = acc;
    __syncthreads();
    // threads t and t + nrhs*q share column c = t % nrhs
    if ((int)threadIdx.x < nrhs) {
        cplx<double> s = {0, 0};
        for (int t = threadIdx.x; t < (int)blockDim.x; t += nrhs) s = s + red[t];
        partial[((int64_t)blockIdx.x * nvec + i) * nrhs + threadIdx.x] = s;
    }
}

__global__ void dots_finish_kernel(const cplx<double> *__restrict__ partial, int nblk, int nvec,
                                   int nrhs, cplx<double> *__restrict__ out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nvec * nrhs) return;
    cplx<double> s = {0, 0};
    for (int b = 0; b < nblk; ++b) s = s + partial[(int64_t)b * nvec * nrhs + q];
    out[q] = s;
}

// w -= sum_i V_i coef[i][c]  (sign = -1) or x += ... (sign = +1)
template <typename T, typename TX>
__global__ void combine_kernel(const cplx<T> *__restrict__ V, int64_t vstride, int nvec,
                               const cplx<double> *__restrict__ coef, cplx<TX> *__restrict__ w,
                               int64_t len, int nrhs, double sign) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += stride) {
        const int c = (int)(k % nrhs);
        cplx<double> s = {0, 0};
        for (int i = 0; i < nvec; ++i) s = s + cvt<double>(V[i * vstride + k]) * coef[i * nrhs + c];
        const cplx<double> o = cvt<double>(w[k]) + sign * s;
        w[k] = cvt<TX>(o);
    }
}

// y[k] = src[k] * scale[c]   (types may differ)
template <typename TS, typename TD>
__global__ void scale_copy_kernel(const cplx<TS> *__restrict__ src, cplx<TD> *__restrict__ dst,
                                  const double *__restrict__ scale, int64_t len, int nrhs) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += stride)
        dst[k] = cvt<TD>(scale[k % nrhs] * cvt<double>(src[k]));
}

// dst[k] = src[k] / |w_c| with |w_c|^2 = nsq[c].re (zero when the norm is 0 or not finite)
template <typename TS, typename TD>
__global__ void normalize_kernel(const cplx<TS> *__restrict__ src, cplx<TD> *__restrict__ dst,
                                 const cplx<double> *__restrict__ nsq, int64_t len, int nrhs) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += stride) {
        const double nn = sqrt(fmax(nsq[k % nrhs].re, 0.0));
        const double s = (nn > 0.0 && isfinite(nn)) ? 1.0 / nn : 0.0;
        dst[k] = cvt<TD>(s * cvt<double>(src[k]));
    }
}

// r = b - r  (in place on r)
template <typename T>
__global__ void bminus_kernel(const cplx<T> *__restrict__ b, cplx<T> *__restrict__ r, int64_t len) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += stride)
        r[k] = b[k] - r[k];
}

// x[k] += scale[c] * d[k]   (x double, d any)
template <typename T>
__global__ void axpy_scaled_kernel(const cplx<T> *__restrict__ d, cplx<double> *__restrict__ x,
                                   const double *__restrict__ scale, int64_t len, int nrhs) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < len; k += stride)
        x[k] = x[k] + scale[k % nrhs] * cvt<double>(d[k]);
}

template <typename T>
class Blas {
   public:
    Blas(int64_t len, int nrhs, int maxvec, hipStream_t st) : len_(len), nrhs_(nrhs), st_(st) {
        bdim_ = 256 - (256 % nrhs);
        nblk_ = (int)std::min<int64_t>(256, std::max<int64_t>(1, ceil_div(len, bdim_)));
        partial_.alloc((size_t)nblk_ * maxvec * nrhs * sizeof(cplx<double>));
        out_.alloc((size_t)maxvec * nrhs * sizeof(cplx<double>));
        coef_.alloc((size_t)maxvec * nrhs * sizeof(cplx<double>));
        scale_.alloc((size_t)nrhs * sizeof(double));
        host_.resize((size_t)maxvec * nrhs);
    }
    // returns host (nvec x nrhs) of V_i^* w
    const std::vector<zd> &dots(const cplx<T> *V, int64_t vstride, int nvec, const cplx<T> *w) {
        hipLaunchKernelGGL(dots_kernel<T>, dim3(nblk_, nvec), dim3(bdim_), 0, st_, V, vstride,
                           nvec, w, len_, nrhs_, partial_.as<cplx<double>>());
        HM_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(dots_finish_kernel, dim3((unsigned)ceil_div(nvec * nrhs_, 256)),
                           dim3(256), 0, st_, partial_.as<cplx<double>>(), nblk_, nvec, nrhs_,
                           out_.as<cplx<double>>());
        HM_HIP_CHECK(hipGetLastError());
        HM_HIP_CHECK(hipMemcpyAsync(host_.data(), out_.p, (size_t)nvec * nrhs_ * sizeof(zd),
                                    hipMemcpyDeviceToHost, st_));
        HM_HIP_CHECK(hipStreamSynchronize(st_));
        return host_;
    }
    // V_i^* w (nvec x nrhs) into the device slot `out` (no host copy)
    void dots_dev(const cplx<T> *V, int64_t vstride, int nvec, const cplx<T> *w,
                  cplx<double> *out) {
        hipLaunchKernelGGL(dots_kernel<T>, dim3(nblk_, nvec), dim3(bdim_), 0, st_, V, vstride,
                           nvec, w, len_, nrhs_, partial_.as<cplx<double>>());
        HM_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(dots_finish_kernel, dim3((unsigned)ceil_div(nvec * nrhs_, 256)),
                           dim3(256), 0, st_, partial_.as<cplx<double>>(), nblk_, nvec, nrhs_, out);
        HM_HIP_CHECK(hipGetLastError());
    }
    // w += sign * sum_i V_i coef[i][c] with device coefficients
    template <typename TX>
    void combine_dev(const cplx<T> *V, int64_t vstride, int nvec, const cplx<double> *coef,
                     cplx<TX> *w, double sign) {
        hipLaunchKernelGGL((combine_kernel<T, TX>), dim3(grid()), dim3(256), 0, st_, V, vstride,
                           nvec, coef, w, len_, nrhs_, sign);
        HM_HIP_CHECK(hipGetLastError());
    }
    // dst = src / |src| per column, |src|^2 from the device slot nsq
    template <typename TS, typename TD>
    void normalize_dev(const cplx<TS> *src, cplx<TD> *dst, const cplx<double> *nsq) {
        hipLaunchKernelGGL((normalize_kernel<TS, TD>), dim3(grid()), dim3(256), 0, st_, src, dst,
                           nsq, len_, nrhs_);
        HM_HIP_CHECK(hipGetLastError());
    }
    std::vector<double> norms(const cplx<T> *w) {
        const auto &h = dots(w, 0, 1, w);
        std::vector<double> n(nrhs_);
        for (int c = 0; c < nrhs_; ++c) n[c] = std::sqrt(std::max(0.0, h[c].real()));
        return n;
    }
    template <typename TX>
    void combine(const cplx<T> *V, int64_t vstride, int nvec, const std::vector<zd> &coef,
                 cplx<TX> *w, double sign) {
        h2d(coef_.p, coef.data(), (size_t)nvec * nrhs_ * sizeof(zd));
        hipLaunchKernelGGL((combine_kernel<T, TX>), dim3(grid()), dim3(256), 0, st_, V, vstride,
                           nvec, coef_.as<cplx<double>>(), w, len_, nrhs_, sign);
        HM_HIP_CHECK(hipGetLastError());
    }
    template <typename TS, typename TD>
    void scale_copy(const cplx<TS> *src, cplx<TD> *dst, const std::vector<double> &s) {
        h2d(scale_.p, s.data(), nrhs_ * sizeof(double));
        hipLaunchKernelGGL((scale_copy_kernel<TS, TD>), dim3(grid()), dim3(256), 0, st_, src, dst,
                           scale_.as<double>(), len_, nrhs_);
        HM_HIP_CHECK(hipGetLastError());
    }
    template <typename TD>
    void axpy_scaled(const cplx<TD> *d, cplx<double> *x, const std::vector<double> &s) {
        h2d(scale_.p, s.data(), nrhs_ * sizeof(double));
        hipLaunchKernelGGL((axpy_scaled_kernel<TD>), dim3(grid()), dim3(256), 0, st_, d, x,
                           scale_.as<double>(), len_, nrhs_);
        HM_HIP_CHECK(hipGetLastError());
    }
    void bminus(const cplx<T> *b, cplx<T> *r) {
        hipLaunchKernelGGL(bminus_kernel<T>, dim3(grid()), dim3(256), 0, st_, b, r, len_);
        HM_HIP_CHECK(hipGetLastError());
    }
    unsigned grid() const { return (unsigned)std::min<int64_t>(2048, ceil_div(len_, 256)); }
    // Small host-to-device copy from pageable memory; completes before returning
    // (the stream is drained first, so earlier kernels reading dst are done too).
    void h2d(void *dst, const void *src, size_t bytes) {
        HM_HIP_CHECK(hipStreamSynchronize(st_));
        HM_HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st_));
        HM_HIP_CHECK(hipStreamSynchronize(st_));
    }

   private:
    int64_t len_;
    int nrhs_, bdim_, nblk_;
    hipStream_t st_;
    DeviceBuf partial_, out_, coef_, scale_;
    std::vector<zd> host_;
};

struct GmresResult {
    int iters = 0, restarts = 0, converged = 0;
    double relres_est = 0;
};

// GMRES in precision T on A x = b (device vectors of type T), x0 = 0.
// tol is relative to |b_c| per column.
template <typename T>
GmresResult gmres_core(const hm_matrix *A, const cplx<T> *b, cplx<T> *x, int nrhs, double tol,
                       int m, int maxit, hipStream_t st) {
    const int64_t n = 3 * A->nx;
    const int64_t len = n * nrhs;
    GmresResult res;
    DeviceBuf Vb, wb;
    Vb.alloc((size_t)(m + 1) * len * sizeof(cplx<T>));
    wb.alloc((size_t)len * sizeof(cplx<T>));
    cplx<T> *V = Vb.as<cplx<T>>(), *w = wb.as<cplx<T>>();
    Blas<T> blas(len, nrhs, m + 1, st);
    // device slots of one Arnoldi step: two CGS passes ((m + 1) x nrhs each) and |w|^2
    DeviceBuf hb_dev;
    hb_dev.alloc((size_t)(2 * (m + 1) + 1) * nrhs * sizeof(cplx<double>));
    cplx<double> *hslots = hb_dev.as<cplx<double>>();
    std::vector<zd> hhost((size_t)(2 * (m + 1) + 1) * nrhs);
    HM_HIP_CHECK(hipMemsetAsync(x, 0, len * sizeof(cplx<T>), st));
    const std::vector<double> bn = blas.norms(b);
    std::vector<char> done(nrhs, 0);
    for (int c = 0; c < nrhs; ++c)
        if (bn[c] == 0.0) done[c] = 1;
    // r0 = b (x0 = 0)
    HM_HIP_CHECK(hipMemcpyAsync(w, b, len * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
    std::vector<zd> H((size_t)(m + 1) * m * nrhs), g((size_t)(m + 1) * nrhs);
    std::vector<zd> cs((size_t)m * nrhs), sn((size_t)m * nrhs);
    std::vector<int> jlast(nrhs, -1);
    auto Hc = [&](int i, int j, int c) -> zd & { return H[((size_t)c * (m + 1) + i) * m + j]; };
    while (true) {
        std::vector<double> beta = blas.norms(w);
        bool all = true;
        for (int c = 0; c < nrhs; ++c) {
            if (!done[c] && beta[c] <= tol * bn[c]) done[c] = 1;
            all = all && done[c];
        }
        res.relres_est = 0;
        for (int c = 0; c < nrhs; ++c)
            if (bn[c] > 0) res.relres_est = std::max(res.relres_est, beta[c] / bn[c]);
        if (all || res.iters >= maxit) break;
        ++res.restarts;
        std::vector<double> inv(nrhs);
        for (int c = 0; c < nrhs; ++c) inv[c] = (beta[c] > 0 && std::isfinite(beta[c])) ? 1.0 / beta[c] : 0.0;
        blas.scale_copy(w, V, inv);
        std::fill(g.begin(), g.end(), zd(0));
        for (int c = 0; c < nrhs; ++c) g[(size_t)c * (m + 1)] = beta[c];
        std::fill(jlast.begin(), jlast.end(), -1);
        std::vector<char> active(nrhs);
        for (int c = 0; c < nrhs; ++c) active[c] = !done[c];
        int j = 0;
        for (; j < m && res.iters < maxit; ++j) {
            cplx<T> *vj = V + (size_t)j * len, *vn = V + (size_t)(j + 1) * len;
            if (hm_matvec(A, vj, w, nrhs, st) != HM_OK) throw StatusError(HM_ERR_HIP, "matvec failed");
            // CGS2 and the normalisation stay on the device; one copy brings the
            // two coefficient passes and |w|^2 to the host for the Givens update.
            const size_t nc = (size_t)(j + 1) * nrhs;
            cplx<double> *c1 = hslots, *c2 = hslots + nc, *nsq = hslots + 2 * nc;
            blas.dots_dev(V, len, j + 1, w, c1);
            blas.combine_dev(V, len, j + 1, c1, w, -1.0);
            blas.dots_dev(V, len, j + 1, w, c2);
            blas.combine_dev(V, len, j + 1, c2, w, -1.0);
            blas.dots_dev(w, 0, 1, w, nsq);
            blas.normalize_dev(w, vn, nsq);
            HM_HIP_CHECK(hipMemcpyAsync(hhost.data(), hslots, (2 * nc + nrhs) * sizeof(zd),
                                        hipMemcpyDeviceToHost, st));
            HM_HIP_CHECK(hipStreamSynchronize(st));
            std::vector<zd> h(nc);
            for (size_t q = 0; q < nc; ++q) h[q] = hhost[q] + hhost[nc + q];
            std::vector<double> hb(nrhs);
            for (int c = 0; c < nrhs; ++c) hb[c] = std::sqrt(std::max(0.0, hhost[2 * nc + c].real()));
            ++res.iters;
            bool cycle_done = true;
            for (int c = 0; c < nrhs; ++c) {
                if (!active[c]) continue;
                for (int i = 0; i <= j; ++i) Hc(i, j, c) = h[(size_t)i * nrhs + c];
                Hc(j + 1, j, c) = hb[c];
                for (int i = 0; i < j; ++i) {
                    const zd c_ = cs[(size_t)c * m + i], s_ = sn[(size_t)c * m + i];
                    const zd a0 = Hc(i, j, c), a1 = Hc(i + 1, j, c);
                    Hc(i, j, c) = std::conj(c_) * a0 + std::conj(s_) * a1;
                    Hc(i + 1, j, c) = -s_ * a0 + c_ * a1;
                }
                const zd a = Hc(j, j, c), bb = Hc(j + 1, j, c);
                const double den = std::sqrt(std::norm(a) + std::norm(bb));
                zd cc = 1, ss = 0;
                if (den > 0) {
                    cc = a / den;
                    ss = bb / den;
                }
                cs[(size_t)c * m + j] = cc;
                sn[(size_t)c * m + j] = ss;
                Hc(j, j, c) = den;
                Hc(j + 1, j, c) = 0;
                zd &g0 = g[(size_t)c * (m + 1) + j];
                zd &g1 = g[(size_t)c * (m + 1) + j + 1];
                const zd gj = g0;
                g0 = std::conj(cc) * gj;
                g1 = -ss * gj;
                jlast[c] = j;
                if (std::abs(g1) <= tol * bn[c] || den == 0) {
                    active[c] = 0;
                } else {
                    cycle_done = false;
                }
            }
            if (cycle_done) {
                ++j;
                break;
            }
        }
        // x += V y per column (back substitution on the rotated Hessenberg)
        const int nv = std::max(1, j);
        std::vector<zd> y((size_t)nv * nrhs, zd(0));
        for (int c = 0; c < nrhs; ++c) {
            const int k = jlast[c];
            for (int i = k; i >= 0; --i) {
                zd s = g[(size_t)c * (m + 1) + i];
                for (int l = i + 1; l <= k; ++l) s -= Hc(i, l, c) * y[(size_t)l * nrhs + c];
                const zd d = Hc(i, i, c);
                y[(size_t)i * nrhs + c] = std::abs(d) > 0 ? s / d : zd(0);
            }
        }
        blas.combine(V, len, nv, y, x, +1.0);
        // explicit residual w = b - A x
        if (hm_matvec(A, x, w, nrhs, st) != HM_OK) throw StatusError(HM_ERR_HIP, "matvec failed");
        blas.bminus(b, w);
    }
    for (int c = 0; c < nrhs; ++c) res.converged += done[c];
    return res;
}

template GmresResult gmres_core<float>(const hm_matrix *, const cplx<float> *, cplx<float> *, int,
                                       double, int, int, hipStream_t);
template GmresResult gmres_core<double>(const hm_matrix *, const cplx<double> *, cplx<double> *,
                                        int, double, int, int, hipStream_t);

}  // namespace hm

using namespace hm;

extern "C" hm_status hm_gmres(const hm_matrix *A, const void *b, void *x, int32_t nrhs, double tol,
                              int32_t restart, int32_t maxit, void *stream, hm_gmres_info *info) {
    try {
        if (!A || !b || !x || nrhs < 1 || nrhs > 256 || !(tol > 0) || restart < 1 || maxit < 1) {
            set_error("invalid GMRES arguments (nrhs in 1..256, tol > 0, restart, maxit >= 1)");
            return HM_ERR_ARG;
        }
        if (A->plan_only) {
            set_error("matrix was built with plan_only");
            return HM_ERR_STATE;
        }
        hipStream_t st = static_cast<hipStream_t>(stream);
        const int64_t len = 3 * A->nx * nrhs;
        hm_gmres_info inf{};
        auto *xd = static_cast<cplx<double> *>(x);
        const auto *bd = static_cast<const cplx<double> *>(b);
        Blas<double> blas(len, nrhs, 1, st);
        const std::vector<double> bn = blas.norms(bd);
        DeviceBuf rbuf;
        rbuf.alloc(len * sizeof(cplx<double>));
        auto *r = rbuf.as<cplx<double>>();
        auto relres_of = [&]() {
            if (hm_residual(A, b, x, r, nrhs, st) != HM_OK)
                throw StatusError(HM_ERR_HIP, "residual failed");
            const std::vector<double> rn = blas.norms(r);
            double worst = 0;
            int ok = 0;
            for (int c = 0; c < nrhs; ++c) {
                const double rr = bn[c] > 0 ? rn[c] / bn[c] : 0.0;
                worst = std::max(worst, rr);
                ok += rr <= tol;
            }
            return std::make_pair(worst, ok);
        };
        if (A->p.prec == HM_C128) {
            int used = 0;
            HM_HIP_CHECK(hipMemsetAsync(x, 0, len * sizeof(cplx<double>), st));
            // Plain FP64 GMRES; if the explicit residual disagrees with the
            // recursive one, continue from the current iterate on the residual.
            DeviceBuf dbuf;
            dbuf.alloc(len * sizeof(cplx<double>));
            for (int round = 0; round < 8 && used < maxit; ++round) {
                auto rr = relres_of();
                inf.relres = rr.first;
                inf.converged = rr.second;
                if (rr.first <= tol) break;
                ++inf.refinements;
                const std::vector<double> rn = blas.norms(r);
                std::vector<double> s(nrhs), sinv(nrhs);
                for (int c = 0; c < nrhs; ++c) {
                    s[c] = rn[c];
                    sinv[c] = rn[c] > 0 ? 1.0 / rn[c] : 0.0;
                }
                blas.scale_copy(r, r, sinv);
                double itol = tol;
                for (int c = 0; c < nrhs; ++c)
                    if (rn[c] > 0) itol = std::min(itol, 0.9 * tol * bn[c] / rn[c]);
                GmresResult g = gmres_core<double>(A, r, dbuf.as<cplx<double>>(), nrhs,
                                                   std::max(itol, 1e-15), restart, maxit - used, st);
                used += g.iters;
                inf.iters += g.iters;
                inf.restarts += g.restarts;
                inf.relres_inner = g.relres_est;
                blas.axpy_scaled(dbuf.as<cplx<double>>(), xd, s);
            }
            inf.refinements = std::max(0, inf.refinements - 1);
            auto rr = relres_of();
            inf.relres = rr.first;
            inf.converged = rr.second;
        } else {
            // FP64 iterative refinement around complex64 inner solves.
            int used = 0;
            HM_HIP_CHECK(hipMemsetAsync(x, 0, len * sizeof(cplx<double>), st));
            DeviceBuf r32, d32;
            r32.alloc(len * sizeof(cplx<float>));
            d32.alloc(len * sizeof(cplx<float>));
            for (int round = 0; round < 30 && used < maxit; ++round) {
                auto rr = relres_of();
                inf.relres = rr.first;
                inf.converged = rr.second;
                if (rr.first <= tol) break;
                ++inf.refinements;
                const std::vector<double> rn = blas.norms(r);
                std::vector<double> s(nrhs), sinv(nrhs);
                for (int c = 0; c < nrhs; ++c) {
                    s[c] = rn[c];
                    sinv[c] = rn[c] > 0 ? 1.0 / rn[c] : 0.0;
                }
                blas.scale_copy(r, r32.as<cplx<float>>(), sinv);
                double itol = 1e-4;
                for (int c = 0; c < nrhs; ++c)
                    if (rn[c] > 0) itol = std::min(itol, std::max(1e-5, 0.5 * tol * bn[c] / rn[c]));
                GmresResult g = gmres_core<float>(A, r32.as<cplx<float>>(), d32.as<cplx<float>>(),
                                                  nrhs, itol, restart, maxit - used, st);
                used += g.iters;
                inf.iters += g.iters;
                inf.restarts += g.restarts;
                inf.relres_inner = g.relres_est;
                blas.axpy_scaled(d32.as<cplx<float>>(), xd, s);
            }
            auto rr = relres_of();
            inf.relres = rr.first;
            inf.converged = rr.second;
        }
        HM_HIP_CHECK(hipStreamSynchronize(st));
        if (info) *info = inf;
        if (inf.relres > tol) {
            set_error("GMRES did not reach tol within maxit");
            return HM_ERR_NOCONV;
        }
        return HM_OK;
    } catch (const StatusError &e) {
        set_error(e.msg);
        return e.status;
    } catch (const HipError &e) {
        set_error(e.msg);
        return HM_ERR_HIP;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return HM_ERR_ALLOC;
    }
}
