// Restarted GMRES on the H-matrix (the iterative solver of Section 3.1).
//
// Reading (the paper names GMRES only): x0 = 0, no preconditioner,
// GMRES(restart) with classical Gram-Schmidt applied twice (CGS2) for the
// Arnoldi step, Givens rotations for the small least-squares problem,
// convergence on the recursive residual, confirmed by an explicit residual
// at every restart.  Within a cycle everything stays on the device: the
// Gram-Schmidt coefficients, the norms, the Hessenberg columns, the
// rotations and the residual vector g.  The host queues step j, then reads
// a 4-byte active count of step j - 1, so it never stalls the GPU; at the
// end of a cycle it copies the triangular system back once and solves it.
// nrhs right-hand sides run as independent GMRES instances in lockstep: one
// multi-column H-matvec per iteration, the BLAS-1 kernels work on all
// columns at once, Hessenberg data per column.
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

// The Arnoldi step is a pair of skinny products with the basis V (nvec
// vectors of len entries, vector i at V + i * vstride): c = V^* w and
// w -= V c.  Both are HBM-bound reads of V; the kernels below split the
// entries into chunks of kGsChunk (64 lanes x kGsE entries per lane) and
// give each wave several vectors, so that a vector of 60k entries still
// spreads over a few thousand waves.
constexpr int kGsE = 2;
constexpr int kGsChunk = 64 * kGsE;
constexpr int kGsIG = 8;          // vectors per wave in gs_dots_kernel
constexpr int kGsWaves = 4096;    // waves per gs_dots_kernel launch (about 4 per SIMD)

// Sum over the lanes of a wave that share lane % nrhs (nrhs a power of two <= 64).
__device__ inline cplx<double> wave_sum_cols(cplx<double> v, int nrhs) {
    for (int o = 32; o >= nrhs; o >>= 1) {
        v.re += __shfl_xor(v.re, o, 64);
        v.im += __shfl_xor(v.im, o, 64);
    }
    return v;
}

// partial[(slot * nvec + i) * nrhs + c] = sum of conj(V_i[k]) w[k] over the
// chunks slot, slot + nslot, ... and the entries k of column c (k % nrhs == c).
// A chunk starts at a multiple of 64 entries, so with nrhs | 64 lane l only
// ever sees column l % nrhs.  Grid: (ceil(nslot / 4), ceil(nvec / kGsIG)).
template <typename T>
__global__ __launch_bounds__(256) void gs_dots_kernel(const cplx<T> *__restrict__ V,
                                                      int64_t vstride, int nvec,
                                                      const cplx<T> *__restrict__ w, int64_t len,
                                                      int nrhs, int nslot,
                                                      cplx<double> *__restrict__ partial) {
    const int lane = threadIdx.x & 63;
    const int slot = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int i0 = blockIdx.y * kGsIG;
    if (slot >= nslot) return;  // per-wave exit: the kernel has no block barrier
    cplx<double> acc[kGsIG];
#pragma unroll
    for (int q = 0; q < kGsIG; ++q) acc[q] = {0, 0};
    const int64_t nch = (len + kGsChunk - 1) / kGsChunk;
    for (int64_t ch = slot; ch < nch; ch += nslot) {
        const int64_t kb = ch * kGsChunk + lane;
        cplx<double> wv[kGsE];
#pragma unroll
        for (int e = 0; e < kGsE; ++e) {
            const int64_t k = kb + 64 * e;
            wv[e] = k < len ? cvt<double>(w[k]) : cplx<double>{0, 0};
        }
#pragma unroll
        for (int q = 0; q < kGsIG; ++q) {
            if (i0 + q >= nvec) break;
            const cplx<T> *v = V + (int64_t)(i0 + q) * vstride;
#pragma unroll
            for (int e = 0; e < kGsE; ++e) {
                const int64_t k = kb + 64 * e;
                if (k < len) acc[q] = acc[q] + cmul(cvt<double>(v[k]), wv[e]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kGsIG; ++q) {
        if (i0 + q >= nvec) break;
        const cplx<double> s = wave_sum_cols(acc[q], nrhs);
        if (lane < nrhs) partial[((int64_t)slot * nvec + i0 + q) * nrhs + lane] = s;
    }
}

// Fallback for nrhs that does not divide 64:
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

// out[q] = sum over s < nslot of partial[s * nq + q]: one wave per output,
// in a fixed order (lane-strided sums, then a butterfly).
__global__ __launch_bounds__(256) void dots_finish_kernel(const cplx<double> *__restrict__ partial,
                                                          int nslot, int nq,
                                                          cplx<double> *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= nq) return;
    cplx<double> s = {0, 0};
    for (int b = lane; b < nslot; b += 64) s = s + partial[(int64_t)b * nq + q];
    s = wave_sum_cols(s, 1);
    if (lane == 0) out[q] = s;
}

// w[k] += sign * sum_i V_i[k] coef[i][k % nrhs].  A block of four waves owns
// kGsChunk entries at a time and splits the vectors between its waves
// (wave q takes i = q, q + 4, ...); waves 1..3 hand their sums to wave 0
// through LDS, so each entry of w is read and written once.
template <typename T, typename TX>
__global__ __launch_bounds__(256) void combine_kernel(const cplx<T> *__restrict__ V,
                                                      int64_t vstride, int nvec,
                                                      const cplx<double> *__restrict__ coef,
                                                      cplx<TX> *__restrict__ w, int64_t len,
                                                      int nrhs, double sign) {
    __shared__ cplx<double> red[3][kGsE][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nch = (len + kGsChunk - 1) / kGsChunk;
    for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
        const int64_t kb = ch * kGsChunk + lane;
        cplx<double> acc[kGsE];
        int col[kGsE];
#pragma unroll
        for (int e = 0; e < kGsE; ++e) {
            acc[e] = {0, 0};
            col[e] = (int)((kb + 64 * e) % nrhs);
        }
#pragma unroll 4
        for (int i = wv; i < nvec; i += 4) {
            const cplx<T> *v = V + (int64_t)i * vstride;
#pragma unroll
            for (int e = 0; e < kGsE; ++e) {
                const int64_t k = kb + 64 * e;
                if (k < len) fma_(acc[e], cvt<double>(v[k]), coef[i * nrhs + col[e]]);
            }
        }
        if (wv > 0) {
#pragma unroll
            for (int e = 0; e < kGsE; ++e) red[wv - 1][e][lane] = acc[e];
        }
        __syncthreads();
        if (wv == 0) {
#pragma unroll
            for (int e = 0; e < kGsE; ++e) {
                const int64_t k = kb + 64 * e;
                if (k < len) {
                    const cplx<double> s = acc[e] + red[0][e][lane] + red[1][e][lane] + red[2][e][lane];
                    w[k] = cvt<TX>(cvt<double>(w[k]) + sign * s);
                }
            }
        }
        __syncthreads();
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

// One Arnoldi step's update of the small least-squares problem, on the
// device so that the host never waits inside a cycle.  One thread per
// right-hand side c (nrhs <= 256, one block).  The Hessenberg column j is
// the sum of the two CGS coefficient passes, its subdiagonal the norm of the
// orthogonalised vector; the earlier rotations are applied, a new rotation
// zeroes the subdiagonal and rotates the residual vector g.  A column stops
// (active = 0) once |g_{j+1}| <= thr_c or the step breaks down.
// Layouts: H[(c * (m + 1) + i) * m + j], cs/sn[c * m + j], g[c * (m + 1) + i];
// slots = [pass 1 ((j + 1) x nrhs) | pass 2 ((j + 1) x nrhs) | |w|^2 (nrhs)].
// status[0] = number of columns still active after this step.
constexpr int kGivensLds = 1024;  // (row, column) entries staged per tile

__global__ __launch_bounds__(256) void givens_kernel(const cplx<double> *__restrict__ slots, int j,
                                                     int m, int nrhs, const double *__restrict__ thr,
                                                     cplx<double> *__restrict__ H,
                                                     cplx<double> *__restrict__ cs,
                                                     cplx<double> *__restrict__ sn,
                                                     cplx<double> *__restrict__ g,
                                                     int *__restrict__ active,
                                                     int *__restrict__ jlast, int *__restrict__ status) {
    // The rotations are a serial chain per column; their inputs (the old
    // rotations and the new Hessenberg entries) are staged through LDS by the
    // whole block, tile by tile, so that the chain itself only waits on LDS.
    __shared__ cplx<double> lc[kGivensLds], ls[kGivensLds], lh[kGivensLds];
    const int c = threadIdx.x;
    const int nc = (j + 1) * nrhs;
    const bool mine = c < nrhs && active[c];
    cplx<double> *Hc = H + (int64_t)(mine ? c : 0) * (m + 1) * m;
    // cur: entry (i, j) of column c after the rotations 0..i-1
    cplx<double> cur = {0, 0};
    if (mine) cur = slots[c] + slots[nc + c];
    const int rows = max(1, kGivensLds / nrhs);
    for (int i0 = 0; i0 < j; i0 += rows) {
        const int ni = min(rows, j - i0);
        __syncthreads();
        for (int t = threadIdx.x; t < ni * nrhs; t += blockDim.x) {
            const int r = t / nrhs, cc = t - r * nrhs, i = i0 + r;
            lc[t] = cs[cc * m + i];
            ls[t] = sn[cc * m + i];
            lh[t] = slots[(i + 1) * nrhs + cc] + slots[nc + (i + 1) * nrhs + cc];
        }
        __syncthreads();
        if (mine) {
            for (int r = 0; r < ni; ++r) {
                const cplx<double> c_ = lc[r * nrhs + c], s_ = ls[r * nrhs + c];
                const cplx<double> a1 = lh[r * nrhs + c];
                Hc[(i0 + r) * m + j] = conj(c_) * cur + conj(s_) * a1;
                cur = c_ * a1 - s_ * cur;
            }
        }
    }
    int still = 0;
    if (mine) {
        const cplx<double> a = cur;
        const double bn = sqrt(fmax(0.0, slots[2 * nc + c].re));
        const double den = sqrt(abs2(a) + bn * bn);
        cplx<double> cc = {1, 0}, ss = {0, 0};
        if (den > 0) {
            cc = (1.0 / den) * a;
            ss = {bn / den, 0.0};
        }
        cs[c * m + j] = cc;
        sn[c * m + j] = ss;
        Hc[j * m + j] = {den, 0};
        Hc[(j + 1) * m + j] = {0, 0};
        cplx<double> *gc = g + (int64_t)c * (m + 1);
        const cplx<double> gj = gc[j];
        gc[j] = conj(cc) * gj;
        const cplx<double> g1 = (-1.0) * (ss * gj);
        gc[j + 1] = g1;
        jlast[c] = j;
        if (sqrt(abs2(g1)) <= thr[c] || den == 0) {
            active[c] = 0;
        } else {
            still = 1;
        }
    }
    const int n = __syncthreads_count(still);
    if (threadIdx.x == 0) status[0] = n;
}

// Page-locked host buffer (hipHostMalloc), so that device-to-host copies of
// small status words stay asynchronous.
template <typename X>
struct PinnedBuf {
    X *p = nullptr;
    explicit PinnedBuf(size_t n) { HM_HIP_CHECK(hipHostMalloc((void **)&p, n * sizeof(X), 0)); }
    PinnedBuf(const PinnedBuf &) = delete;
    PinnedBuf &operator=(const PinnedBuf &) = delete;
    ~PinnedBuf() {
        if (p) (void)hipHostFree(p);
    }
};

template <typename T>
class Blas {
   public:
    Blas(int64_t len, int nrhs, int maxvec, hipStream_t st) : len_(len), nrhs_(nrhs), st_(st) {
        bdim_ = 256 - (256 % nrhs);
        nblk_ = (int)std::min<int64_t>(256, std::max<int64_t>(1, ceil_div(len, bdim_)));
        chunked_ = nrhs <= 64 && (64 % nrhs) == 0;
        size_t slots = (size_t)nblk_ * maxvec;
        if (chunked_)
            for (int nv = 1; nv <= maxvec; ++nv) slots = std::max(slots, (size_t)nslot(nv) * nv);
        partial_.alloc(slots * nrhs * sizeof(cplx<double>));
        out_.alloc((size_t)maxvec * nrhs * sizeof(cplx<double>));
        coef_.alloc((size_t)maxvec * nrhs * sizeof(cplx<double>));
        scale_.alloc((size_t)nrhs * sizeof(double));
        host_.resize((size_t)maxvec * nrhs);
    }
    // returns host (nvec x nrhs) of V_i^* w
    const std::vector<zd> &dots(const cplx<T> *V, int64_t vstride, int nvec, const cplx<T> *w) {
        dots_dev(V, vstride, nvec, w, out_.as<cplx<double>>());
        HM_HIP_CHECK(hipMemcpyAsync(host_.data(), out_.p, (size_t)nvec * nrhs_ * sizeof(zd),
                                    hipMemcpyDeviceToHost, st_));
        HM_HIP_CHECK(hipStreamSynchronize(st_));
        return host_;
    }
    // V_i^* w (nvec x nrhs) into the device slot `out` (no host copy)
    void dots_dev(const cplx<T> *V, int64_t vstride, int nvec, const cplx<T> *w,
                  cplx<double> *out) {
        int ns = nblk_;
        if (chunked_) {
            ns = nslot(nvec);
            hipLaunchKernelGGL(gs_dots_kernel<T>,
                               dim3((unsigned)ceil_div(ns, 4), (unsigned)ceil_div(nvec, kGsIG)),
                               dim3(256), 0, st_, V, vstride, nvec, w, len_, nrhs_, ns,
                               partial_.as<cplx<double>>());
        } else {
            hipLaunchKernelGGL(dots_kernel<T>, dim3(nblk_, nvec), dim3(bdim_), 0, st_, V, vstride,
                               nvec, w, len_, nrhs_, partial_.as<cplx<double>>());
        }
        HM_HIP_CHECK(hipGetLastError());
        const int nq = nvec * nrhs_;
        hipLaunchKernelGGL(dots_finish_kernel, dim3((unsigned)ceil_div(nq, 4)), dim3(256), 0, st_,
                           partial_.as<cplx<double>>(), ns, nq, out);
        HM_HIP_CHECK(hipGetLastError());
    }
    // w += sign * sum_i V_i coef[i][c] with device coefficients
    template <typename TX>
    void combine_dev(const cplx<T> *V, int64_t vstride, int nvec, const cplx<double> *coef,
                     cplx<TX> *w, double sign) {
        hipLaunchKernelGGL((combine_kernel<T, TX>), dim3(combine_grid()), dim3(256), 0, st_, V,
                           vstride, nvec, coef, w, len_, nrhs_, sign);
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
        hipLaunchKernelGGL((combine_kernel<T, TX>), dim3(combine_grid()), dim3(256), 0, st_, V,
                           vstride, nvec, coef_.as<cplx<double>>(), w, len_, nrhs_, sign);
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
    unsigned combine_grid() const {
        return (unsigned)std::min<int64_t>(16384, ceil_div(len_, kGsChunk));
    }
    // chunk slots of one gs_dots_kernel launch over nvec vectors
    int nslot(int nvec) const {
        const int64_t nch = ceil_div(len_, kGsChunk);
        const int64_t groups = ceil_div(nvec, kGsIG);
        return (int)std::max<int64_t>(1, std::min<int64_t>(nch, kGsWaves / groups));
    }
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
    bool chunked_;
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
    // the small least-squares problem of every column lives on the device
    const size_t nH = (size_t)(m + 1) * m * nrhs, ng = (size_t)(m + 1) * nrhs;
    DeviceBuf Hd, csd, snd, gd, thrd, actd, jld, std_;
    Hd.alloc(nH * sizeof(cplx<double>));
    csd.alloc((size_t)m * nrhs * sizeof(cplx<double>));
    snd.alloc((size_t)m * nrhs * sizeof(cplx<double>));
    gd.alloc(ng * sizeof(cplx<double>));
    thrd.alloc(nrhs * sizeof(double));
    actd.alloc(nrhs * sizeof(int));
    jld.alloc(nrhs * sizeof(int));
    std_.alloc((size_t)m * sizeof(int));
    PinnedBuf<int> hstat(m);
    ScopedEvent ev[2];
    HM_HIP_CHECK(hipMemsetAsync(x, 0, len * sizeof(cplx<T>), st));
    const std::vector<double> bn = blas.norms(b);
    std::vector<char> done(nrhs, 0);
    for (int c = 0; c < nrhs; ++c)
        if (bn[c] == 0.0) done[c] = 1;
    std::vector<double> thr(nrhs);
    for (int c = 0; c < nrhs; ++c) thr[c] = tol * bn[c];
    blas.h2d(thrd.p, thr.data(), nrhs * sizeof(double));
    // r0 = b (x0 = 0)
    HM_HIP_CHECK(hipMemcpyAsync(w, b, len * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
    std::vector<zd> H(nH), g(ng);
    std::vector<int> jlast(nrhs), act(nrhs);
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
        for (int c = 0; c < nrhs; ++c) {
            g[(size_t)c * (m + 1)] = beta[c];
            act[c] = !done[c];
            jlast[c] = -1;
        }
        blas.h2d(gd.p, g.data(), ng * sizeof(zd));
        blas.h2d(actd.p, act.data(), nrhs * sizeof(int));
        blas.h2d(jld.p, jlast.data(), nrhs * sizeof(int));
        // Arnoldi steps are queued one ahead of the host: step j is queued,
        // then the host reads the active count of step j - 1 and stops the
        // cycle when it is zero (step j then finds no active column and
        // changes nothing in the least-squares data).
        const int jmax = (int)std::min<int64_t>(m, (int64_t)maxit - res.iters);
        for (int j = 0; j < jmax; ++j) {
            cplx<T> *vj = V + (size_t)j * len, *vn = V + (size_t)(j + 1) * len;
            if (hm_matvec(A, vj, w, nrhs, st) != HM_OK) throw StatusError(HM_ERR_HIP, "matvec failed");
            const size_t nc = (size_t)(j + 1) * nrhs;
            cplx<double> *c1 = hslots, *c2 = hslots + nc, *nsq = hslots + 2 * nc;
            blas.dots_dev(V, len, j + 1, w, c1);
            blas.combine_dev(V, len, j + 1, c1, w, -1.0);
            blas.dots_dev(V, len, j + 1, w, c2);
            blas.combine_dev(V, len, j + 1, c2, w, -1.0);
            blas.dots_dev(w, 0, 1, w, nsq);
            blas.normalize_dev(w, vn, nsq);
            hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(256), 0, st, hslots, j, m, nrhs,
                               thrd.as<double>(), Hd.as<cplx<double>>(), csd.as<cplx<double>>(),
                               snd.as<cplx<double>>(), gd.as<cplx<double>>(), actd.as<int>(),
                               jld.as<int>(), std_.as<int>() + j);
            HM_HIP_CHECK(hipGetLastError());
            HM_HIP_CHECK(hipMemcpyAsync(hstat.p + j, std_.as<int>() + j, sizeof(int),
                                        hipMemcpyDeviceToHost, st));
            HM_HIP_CHECK(hipEventRecord(ev[j & 1].e, st));
            if (j >= 1) {
                HM_HIP_CHECK(hipEventSynchronize(ev[(j - 1) & 1].e));
                if (hstat.p[j - 1] == 0) break;
            }
        }
        HM_HIP_CHECK(hipMemcpyAsync(H.data(), Hd.p, nH * sizeof(zd), hipMemcpyDeviceToHost, st));
        HM_HIP_CHECK(hipMemcpyAsync(g.data(), gd.p, ng * sizeof(zd), hipMemcpyDeviceToHost, st));
        HM_HIP_CHECK(hipMemcpyAsync(jlast.data(), jld.p, nrhs * sizeof(int), hipMemcpyDeviceToHost, st));
        HM_HIP_CHECK(hipStreamSynchronize(st));
        // steps with at least one active column
        int steps = 0;
        for (int c = 0; c < nrhs; ++c) steps = std::max(steps, jlast[c] + 1);
        res.iters += steps;
        // x += V y per column (back substitution on the rotated Hessenberg)
        const int nv = std::max(1, steps);
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
        if (steps == 0) break;  // every column was inactive: nothing left to do
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
