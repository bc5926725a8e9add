// Randomized low-rank approximation (the remark closing Section 2.3: blocks of
// the double-layer kernel T whose 3x3 sub-blocks are all singular, where the
// vector ACA can only fall back to rank-deficient pivots).  The range finder
// of Liberty, Woolfe, Martinsson, Rokhlin and Tygert (2007):
//   Y = A Omega        Omega: 3n x k complex Gaussian (counter-based SplitMix64
//                      of Steele, Lea and Flood 2014, Box-Muller), FP64 matrix cores
//   Q = orth(Y)        classical Gram-Schmidt with one reorthogonalisation, FP64
//   B^* = A^* Q        FP64 matrix cores
// with |A - Q Q^* A|_F^2 = |A|_F^2 - |B|_F^2 deciding whether k suffices (the
// host doubles k for the blocks that miss (eps / 2)^2 |A|_F^2).  The block A is
// evaluated in full beforehand (near-field kernel over column slices), and the
// pair (Q, B^*) leaves as ACA-layout factors for the usual QR + SVD
// recompression, which truncates them to eps.
#include <algorithm>
#include <map>

#include "internal.hpp"
#include "mfma_gemm.hpp"
#include "rng.hpp"

namespace hm {

// Omega (rows x k, row-major): entry e = r k + c is gauss_at(seed, e).
__global__ void rs_omega_kernel(cplx<double> *__restrict__ om, int64_t rows, int k,
                                uint64_t seed) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * k) return;
    om[e] = gauss_at(seed, (uint64_t)e);
}

__device__ inline double block_sum256(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double t = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return t;
}

// Y[row0 .. row0 + 64) = A[row0 .. , :] Omega, and |A|_F^2 over those rows.
template <typename R>
__global__ void __launch_bounds__(256) rs_y_kernel(const RsBlk *__restrict__ blks,
                                                   const RsTask *__restrict__ tasks,
                                                   const cplx<R> *__restrict__ dense,
                                                   const cplx<double> *__restrict__ om,
                                                   cplx<double> *__restrict__ fp,
                                                   double *__restrict__ part) {
    __shared__ double sh[4];
    const RsTask t = tasks[blockIdx.x];
    const RsBlk b = blks[t.blk];
    const int64_t rows = 3 * (int64_t)b.m, cols = 3 * (int64_t)b.n;
    const int k = b.k;
    const cplx<R> *A = dense + b.aoff;
    const cplx<double> *Om = om + b.omoff;
    cplx<double> *Y = fp + b.yoff;
    const int64_t row0 = t.row0;
    const int nr = (int)min<int64_t>(64, rows - row0);
    mfma_gemm(
        nr, k, (int)cols, [&](int i, int q) { return cvt<double>(A[(int64_t)q * rows + row0 + i]); },
        [&](int q, int c) { return Om[(int64_t)q * k + c]; },
        [&](int i, int c, cplx<double> v) { Y[(int64_t)c * rows + row0 + i] = v; });
    double s = 0;
    for (int64_t q = threadIdx.x; q < (int64_t)nr * cols; q += blockDim.x)
        s += abs2(cvt<double>(A[(q / nr) * rows + row0 + q % nr]));
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// In place Q = orth(Y), one workgroup per block: classical Gram-Schmidt with
// one reorthogonalisation per column; a column whose norm falls below 1e-12 of
// its norm before the projections is numerically dependent and becomes zero.
template <int NT>
__global__ void __launch_bounds__(NT) rs_orth_kernel(const RsBlk *__restrict__ blks,
                                                     cplx<double> *__restrict__ fp) {
    constexpr int NW = NT / 64;
    __shared__ cplx<double> coef[kRsMaxK];
    __shared__ double sh[NW];
    // block-wide sum, partial sums added in wave order
    auto bsum = [&](double v) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
        __syncthreads();
        double t = 0;
        for (int w = 0; w < NW; ++w) t += sh[w];
        __syncthreads();
        return t;
    };
    const RsBlk b = blks[blockIdx.x];
    const int64_t rows = 3 * (int64_t)b.m;
    const int k = b.k;
    cplx<double> *Y = fp + b.yoff;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int j = 0; j < k; ++j) {
        cplx<double> *yj = Y + (int64_t)j * rows;
        double n0 = 0;
        for (int64_t r = tid; r < rows; r += NT) n0 += abs2(yj[r]);
        n0 = NT == 256 ? block_sum256(n0, sh) : bsum(n0);
        for (int pass = 0; pass < 2; ++pass) {
            for (int i = wave; i < j; i += NW) {
                const cplx<double> *qi = Y + (int64_t)i * rows;
                double dr = 0, di = 0;
                for (int64_t r = lane; r < rows; r += 64) {
                    const cplx<double> v = cmul(qi[r], yj[r]);
                    dr += v.re;
                    di += v.im;
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    dr += __shfl_xor(dr, o, 64);
                    di += __shfl_xor(di, o, 64);
                }
                if (lane == 0) coef[i] = {dr, di};
            }
            __syncthreads();
            for (int64_t r = tid; r < rows; r += NT) {
                cplx<double> acc = yj[r];
                for (int i = 0; i < j; ++i) acc = acc - coef[i] * Y[(int64_t)i * rows + r];
                yj[r] = acc;
            }
            __syncthreads();
        }
        double n1 = 0;
        for (int64_t r = tid; r < rows; r += NT) n1 += abs2(yj[r]);
        n1 = NT == 256 ? block_sum256(n1, sh) : bsum(n1);
        const double sc = (n1 > 1e-24 * n0 && n1 > 0.0) ? 1.0 / sqrt(n1) : 0.0;
        for (int64_t r = tid; r < rows; r += NT) yj[r] = sc * yj[r];
        __syncthreads();
    }
}

// B^*[row0 .. row0 + 64) = (A^* Q)[row0 .., :], and |B|_F^2 over those rows.
template <typename R>
__global__ void __launch_bounds__(256) rs_b_kernel(const RsBlk *__restrict__ blks,
                                                   const RsTask *__restrict__ tasks,
                                                   const cplx<R> *__restrict__ dense,
                                                   cplx<double> *__restrict__ fp,
                                                   double *__restrict__ part) {
    __shared__ double sh[4];
    const RsTask t = tasks[blockIdx.x];
    const RsBlk b = blks[t.blk];
    const int64_t rows = 3 * (int64_t)b.m, cols = 3 * (int64_t)b.n;
    const int k = b.k;
    const cplx<R> *A = dense + b.aoff;
    const cplx<double> *Q = fp + b.yoff;
    cplx<double> *Bh = fp + b.boff;
    const int64_t row0 = t.row0;
    const int nr = (int)min<int64_t>(64, cols - row0);
    double s = 0;
    mfma_gemm(
        nr, k, (int)rows,
        [&](int jj, int i) { return conj(cvt<double>(A[(row0 + jj) * rows + i])); },
        [&](int i, int c) { return Q[(int64_t)c * rows + i]; },
        [&](int jj, int c, cplx<double> v) {
            Bh[(int64_t)c * cols + row0 + jj] = v;
            s += abs2(v);
        });
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Q -> U (3m x k) and B^* -> V (3n x k), column-major in the factor scratch,
// rounded to the storage type.
template <typename R>
__global__ void __launch_bounds__(256) rs_store_kernel(const RsBlk *__restrict__ blks,
                                                       const cplx<double> *__restrict__ fp,
                                                       cplx<R> *__restrict__ fac) {
    const RsBlk b = blks[blockIdx.y];
    const int64_t nu = 3 * (int64_t)b.m * b.k, nv = 3 * (int64_t)b.n * b.k;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nu + nv;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < nu)
            fac[b.uoff + e] = cvt<R>(fp[b.yoff + e]);
        else
            fac[b.voff + (e - nu)] = cvt<R>(fp[b.boff + (e - nu)]);
    }
}

template <typename R>
void run_rsvd(const Geometry &g, const GreenParams<R> &gp, std::vector<RsIn> &blk, double eps,
              int k0, uint64_t seed, std::unique_ptr<DeviceBuf> &factors, hipStream_t st) {
    const size_t nb = blk.size();
    if (nb == 0) return;
    // the blocks in full, evaluated by the near-field kernel over column slices
    std::vector<DenseBlk> tiles;
    int64_t dlen = 0;
    for (auto &b : blk) {
        b.aoff = dlen;
        const int64_t ld = 3 * (int64_t)b.m;
        const int32_t slice = std::max<int32_t>(1, (int32_t)(4096 / std::max<int32_t>(1, b.m)));
        for (int32_t j0 = 0; j0 < b.n; j0 += slice)
            tiles.push_back({dlen + 3 * (int64_t)j0 * ld, b.rb, b.m, b.cb + j0,
                             std::min(slice, b.n - j0), (int32_t)ld, 0});
        dlen += ld * 3 * (int64_t)b.n;
    }
    DeviceBuf d_dense, d_tiles, d_err;
    d_dense.alloc(std::max<int64_t>(dlen, 1) * sizeof(cplx<R>));
    d_tiles.alloc(tiles.size() * sizeof(DenseBlk));
    HM_HIP_CHECK(hipMemcpyAsync(d_tiles.p, tiles.data(), tiles.size() * sizeof(DenseBlk),
                                hipMemcpyHostToDevice, st));
    d_err.alloc(sizeof(int32_t));
    HM_HIP_CHECK(hipMemsetAsync(d_err.p, 0, sizeof(int32_t), st));
    launch_nearfield<R>(g, gp, d_tiles.as<DenseBlk>(), (int32_t)tiles.size(),
                        d_dense.as<cplx<R>>(), R(0), R(0), d_err.as<int32_t>(), st, false);
    int32_t nerr = 0;
    HM_HIP_CHECK(hipMemcpyAsync(&nerr, d_err.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HM_HIP_CHECK(hipStreamSynchronize(st));
    if (nerr) throw StatusError(HM_ERR_SINGULAR, "coincident points in an admissible block");
    // samples: k0, doubled for the blocks whose range misses (eps / 2) |A|_F
    std::vector<int32_t> k(nb);
    for (size_t q = 0; q < nb; ++q)
        k[q] = std::min({k0, 3 * blk[q].m, 3 * blk[q].n, kRsMaxK});
    std::vector<uint8_t> done(nb, 0);
    std::vector<double> na2(nb, 0.0), nbq2(nb, 0.0);
    std::unique_ptr<DeviceBuf> fp;   // Y/Q and B^* of the accepted attempt of every block
    std::vector<RsBlk> final_desc(nb);
    std::vector<std::unique_ptr<DeviceBuf>> keep;   // buffers holding accepted blocks
    for (int attempt = 0;; ++attempt) {
        std::vector<size_t> act;
        for (size_t q = 0; q < nb; ++q)
            if (!done[q]) act.push_back(q);
        if (act.empty()) break;
        // test matrices for every distinct k of this attempt (shared by the blocks)
        std::map<int32_t, int64_t> om_off;
        int64_t omlen = 0, nmax = 0;
        for (size_t q : act) nmax = std::max<int64_t>(nmax, 3 * (int64_t)blk[q].n);
        for (size_t q : act)
            if (!om_off.count(k[q])) {
                om_off[k[q]] = omlen;
                omlen += nmax * k[q];
            }
        DeviceBuf d_om;
        d_om.alloc(omlen * sizeof(cplx<double>));
        for (auto &kv : om_off) {
            const int64_t cnt = nmax * kv.first;
            hipLaunchKernelGGL(rs_omega_kernel, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st,
                               d_om.as<cplx<double>>() + kv.second, nmax, kv.first, seed);
        }
        HM_HIP_CHECK(hipGetLastError());
        std::vector<RsBlk> desc(act.size());
        std::vector<RsTask> ty, tb;
        std::vector<int64_t> ty0(act.size() + 1), tb0(act.size() + 1);
        int64_t flen = 0;
        for (size_t a = 0; a < act.size(); ++a) {
            const RsIn &in = blk[act[a]];
            RsBlk &d = desc[a];
            d.aoff = in.aoff;
            d.omoff = om_off[k[act[a]]];
            d.m = in.m;
            d.n = in.n;
            d.k = k[act[a]];
            d.yoff = flen;
            flen += 3 * (int64_t)in.m * d.k;
            d.boff = flen;
            flen += 3 * (int64_t)in.n * d.k;
            d.uoff = d.voff = 0;
            ty0[a] = (int64_t)ty.size();
            for (int32_t r0 = 0; r0 < 3 * in.m; r0 += 64) ty.push_back({(int32_t)a, r0, 0, 0});
            tb0[a] = (int64_t)tb.size();
            for (int32_t r0 = 0; r0 < 3 * in.n; r0 += 64) tb.push_back({(int32_t)a, r0, 0, 0});
        }
        ty0[act.size()] = (int64_t)ty.size();
        tb0[act.size()] = (int64_t)tb.size();
        auto buf = std::make_unique<DeviceBuf>();
        buf->alloc(std::max<int64_t>(flen, 1) * sizeof(cplx<double>));
        DeviceBuf d_desc, d_ty, d_tb, d_py, d_pb;
        auto put = [&](DeviceBuf &dv, const auto &v) {
            using E = typename std::decay_t<decltype(v)>::value_type;
            dv.alloc(std::max<size_t>(v.size(), 1) * sizeof(E));
            HM_HIP_CHECK(hipMemcpyAsync(dv.p, v.data(), v.size() * sizeof(E),
                                        hipMemcpyHostToDevice, st));
        };
        put(d_desc, desc);
        put(d_ty, ty);
        put(d_tb, tb);
        d_py.alloc(ty.size() * sizeof(double));
        d_pb.alloc(tb.size() * sizeof(double));
        hipLaunchKernelGGL(rs_y_kernel<R>, dim3((unsigned)ty.size()), dim3(256), 0, st,
                           d_desc.as<RsBlk>(), d_ty.as<RsTask>(), d_dense.as<cplx<R>>(),
                           d_om.as<cplx<double>>(), buf->as<cplx<double>>(), d_py.as<double>());
        hipLaunchKernelGGL(rs_orth_kernel<256>, dim3((unsigned)act.size()), dim3(256), 0, st,
                           d_desc.as<RsBlk>(), buf->as<cplx<double>>());
        hipLaunchKernelGGL(rs_b_kernel<R>, dim3((unsigned)tb.size()), dim3(256), 0, st,
                           d_desc.as<RsBlk>(), d_tb.as<RsTask>(), d_dense.as<cplx<R>>(),
                           buf->as<cplx<double>>(), d_pb.as<double>());
        HM_HIP_CHECK(hipGetLastError());
        std::vector<double> py(ty.size()), pb(tb.size());
        HM_HIP_CHECK(hipMemcpyAsync(py.data(), d_py.p, py.size() * sizeof(double),
                                    hipMemcpyDeviceToHost, st));
        HM_HIP_CHECK(hipMemcpyAsync(pb.data(), d_pb.p, pb.size() * sizeof(double),
                                    hipMemcpyDeviceToHost, st));
        HM_HIP_CHECK(hipStreamSynchronize(st));
        bool any_kept = false;
        for (size_t a = 0; a < act.size(); ++a) {
            const size_t q = act[a];
            double sa = 0, sb = 0;   // in task order: the same sums on every run
            for (int64_t t = ty0[a]; t < ty0[a + 1]; ++t) sa += py[t];
            for (int64_t t = tb0[a]; t < tb0[a + 1]; ++t) sb += pb[t];
            const double err2 = std::max(sa - sb, 0.0);
            const int32_t kmax = std::min({3 * blk[q].m, 3 * blk[q].n, kRsMaxK});
            if (err2 <= 0.25 * eps * eps * sa || k[q] >= kmax) {
                done[q] = 1;
                na2[q] = sa;
                nbq2[q] = sb;
                final_desc[q] = desc[a];   // its offsets point into buf
                blk[q].buf = (int32_t)keep.size();
                any_kept = true;
            } else {
                k[q] = std::min(2 * k[q], kmax);
            }
        }
        if (any_kept) keep.push_back(std::move(buf));
    }
    // the accepted (Q, B^*) of every block into one factor scratch, ACA layout
    int64_t len = 0;
    for (size_t q = 0; q < nb; ++q) {
        blk[q].k = final_desc[q].k;
        blk[q].uoff = len;
        len += 3 * (int64_t)blk[q].m * blk[q].k;
        blk[q].voff = len;
        len += 3 * (int64_t)blk[q].n * blk[q].k;
        blk[q].range_err2 = std::max(na2[q] - nbq2[q], 0.0);
        blk[q].norm2 = na2[q];
    }
    factors = std::make_unique<DeviceBuf>();
    factors->alloc(std::max<int64_t>(len, 1) * sizeof(cplx<R>));
    for (size_t kb = 0; kb < keep.size(); ++kb) {
        std::vector<RsBlk> sd;
        for (size_t q = 0; q < nb; ++q)
            if (blk[q].buf == (int32_t)kb) {
                RsBlk d = final_desc[q];
                d.uoff = blk[q].uoff;
                d.voff = blk[q].voff;
                sd.push_back(d);
            }
        if (sd.empty()) continue;
        DeviceBuf d_sd;
        d_sd.alloc(sd.size() * sizeof(RsBlk));
        HM_HIP_CHECK(hipMemcpyAsync(d_sd.p, sd.data(), sd.size() * sizeof(RsBlk),
                                    hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(rs_store_kernel<R>, dim3(64, (unsigned)sd.size()), dim3(256), 0, st,
                           d_sd.as<RsBlk>(), keep[kb]->as<cplx<double>>(),
                           factors->as<cplx<R>>());
        HM_HIP_CHECK(hipGetLastError());
        HM_HIP_CHECK(hipStreamSynchronize(st));
    }
}

void launch_orth(const RsBlk *d_blk, int32_t nblk, cplx<double> *base, hipStream_t st, bool wide) {
    if (nblk <= 0) return;
    if (wide)
        hipLaunchKernelGGL(rs_orth_kernel<1024>, dim3((unsigned)nblk), dim3(1024), 0, st, d_blk, base);
    else
        hipLaunchKernelGGL(rs_orth_kernel<256>, dim3((unsigned)nblk), dim3(256), 0, st, d_blk, base);
    HM_HIP_CHECK(hipGetLastError());
}

template void run_rsvd<float>(const Geometry &, const GreenParams<float> &, std::vector<RsIn> &,
                              double, int, uint64_t, std::unique_ptr<DeviceBuf> &, hipStream_t);
template void run_rsvd<double>(const Geometry &, const GreenParams<double> &,
                               std::vector<RsIn> &, double, int, uint64_t,
                               std::unique_ptr<DeviceBuf> &, hipStream_t);

}  // namespace hm
