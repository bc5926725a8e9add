// H-matrix-vector product (Section 3.1): y = sum over leaf blocks of the
// dense tile times x_sigma, or U (V^* x_sigma) for low-rank blocks.
//
// Storage: dense tiles and U column-major with the padded leaf-segment row
// layout (even leading dimension, every leaf segment starting on an even
// row); V stored row-major (3n x r, row stride r rounded up to even).
// Three passes, no atomics, every output row written exactly once:
//   gather   x (original order, one column) -> xc (column-cluster order)
//   project  t_b = V_b^* xc[sigma_b]: one wave per (block, group of up to 64
//            columns); lanes own columns (floor(64/r) row groups of r lanes
//            when r < 64), so each iteration of the wave reads one contiguous
//            segment of the row-major V; the row groups are summed in LDS
//   accum    one workgroup per leaf row cluster L: the sum over the dense
//            tiles of L and over the rows of every low-rank U whose row
//            cluster contains L; lanes own rows (complex64: row pairs read
//            with one 16-byte load), waves split the task list, 8-way
//            unrolled column loops keep loads in flight, LDS combines
//            the waves, and the result is scattered to original order (or
//            subtracted from b for the FP64 residual).
// S is the storage real type, A the accumulation real type.
#include <algorithm>
#include <mutex>

#include "internal.hpp"

namespace hm {

constexpr int kWave = 64;

// Stored factors are streamed once per product: non-temporal loads keep them
// from displacing the reused x and t vectors in the caches.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ inline float4 ld_stream(const float4 *p) {
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline cplx<float> ld_stream(const cplx<float> *p) {
    const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(p));
    return {v.x, v.y};
}
__device__ inline cplx<double> ld_stream(const cplx<double> *p) {
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
    return {v.x, v.y};
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
                                                      const ProjTask *__restrict__ ptasks,
                                                      int32_t ntasks,
                                                      const cplx<S> *__restrict__ fac,
                                                      const cplx<A> *__restrict__ xc,
                                                      cplx<A> *__restrict__ t,
                                                      cplx<A> *__restrict__ tpart) {
    // complex64: each lane owns a column pair (one 16-byte load per row; the
    // even row stride and zero pad column keep loads aligned and in bounds)
    constexpr bool PAIR = sizeof(S) == 4 && sizeof(A) == 4;
    constexpr int CPL = PAIR ? 2 : 1;   // columns per lane
    __shared__ cplx<A> part[256 * CPL];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t ti = blockIdx.x * (blockDim.x / kWave) + wave;
    const bool live = ti < ntasks;
    cplx<A> acc[CPL];
#pragma unroll
    for (int h = 0; h < CPL; ++h) acc[h] = {A(0), A(0)};
    int width = 1, G = 1, lw = 1;
    LowRankBlk b;
    ProjTask pt = {0, 0, 0, 0, -1, 0};
    if (live) {
        pt = ptasks[ti];
        b = blk[pt.blk];
        width = min(64, b.r - pt.col0);
        lw = (width + CPL - 1) / CPL;   // lanes per row
        // G row groups of lw lanes: for a fixed iteration the wave reads G
        // consecutive rows of the row-major V, i.e. one contiguous segment.
        G = kWave / lw;
        const int g = lane / lw, c = lane - g * lw;
        if (g < G) {
            const int32_t rows = pt.nrows;
            const int64_t ldv = b.ldv;
            const cplx<S> *v = fac + b.voff + (int64_t)pt.row0 * ldv + pt.col0 + CPL * c;
            const cplx<A> *xs = xc + 3 * (int64_t)b.cb + pt.row0;
            int32_t i = g;
            if constexpr (PAIR) {
                for (; i + 7 * G < rows; i += 8 * G) {
                    float4 vv[8];
                    cplx<A> xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        vv[u] = ld_stream(reinterpret_cast<const float4 *>(v + (int64_t)(i + u * G) * ldv));
                        xv[u] = xs[i + u * G];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        // conj(v) * x for both columns
                        acc[0].re += vv[u].x * xv[u].re + vv[u].y * xv[u].im;
                        acc[0].im += vv[u].x * xv[u].im - vv[u].y * xv[u].re;
                        acc[1].re += vv[u].z * xv[u].re + vv[u].w * xv[u].im;
                        acc[1].im += vv[u].z * xv[u].im - vv[u].w * xv[u].re;
                    }
                }
                for (; i < rows; i += G) {
                    const float4 vv = ld_stream(reinterpret_cast<const float4 *>(v + (int64_t)i * ldv));
                    const cplx<A> xv = xs[i];
                    acc[0].re += vv.x * xv.re + vv.y * xv.im;
                    acc[0].im += vv.x * xv.im - vv.y * xv.re;
                    acc[1].re += vv.z * xv.re + vv.w * xv.im;
                    acc[1].im += vv.z * xv.im - vv.w * xv.re;
                }
            } else {
                for (; i + 7 * G < rows; i += 8 * G) {
                    cplx<S> vv[8];
                    cplx<A> xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        vv[u] = ld_stream(v + (int64_t)(i + u * G) * ldv);
                        xv[u] = xs[i + u * G];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const cplx<A> a = cvt<A>(vv[u]);
                        acc[0].re += a.re * xv[u].re + a.im * xv[u].im;
                        acc[0].im += a.re * xv[u].im - a.im * xv[u].re;
                    }
                }
                for (; i < rows; i += G) {
                    const cplx<A> a = cvt<A>(ld_stream(v + (int64_t)i * ldv));
                    const cplx<A> xv = xs[i];
                    acc[0].re += a.re * xv.re + a.im * xv.im;
                    acc[0].im += a.re * xv.im - a.im * xv.re;
                }
            }
        }
    }
    // sum the G row groups of each column through LDS (per-wave region);
    // part index (wave, lane) * CPL + h holds column CPL * (lane % lw) + h of row group lane / lw
#pragma unroll
    for (int h = 0; h < CPL; ++h) part[threadIdx.x * CPL + h] = acc[h];
    __syncthreads();
    if (live && lane < width) {
        const int cl = lane / CPL, h = lane % CPL;   // column `lane` lives in lane cl, slot h
        cplx<A> s = {A(0), A(0)};
        for (int q = 0; q < G; ++q) s = s + part[(wave * kWave + q * lw + cl) * CPL + h];
        if (pt.slot < 0)
            t[b.toff + pt.col0 + lane] = s;
        else
            tpart[(int64_t)pt.slot * kWave + lane] = s;
    }
}

// t = sum of the row-chunk partial projections (fixed order: deterministic).
template <typename A>
__global__ void project_reduce_kernel(const LowRankBlk *__restrict__ blk,
                                      const ProjReduce *__restrict__ red, int32_t nred,
                                      const cplx<A> *__restrict__ tpart, cplx<A> *__restrict__ t) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t k = blockIdx.x * (blockDim.x / kWave) + wave;
    if (k >= nred) return;
    const ProjReduce pr = red[k];
    const LowRankBlk b = blk[pr.blk];
    if (lane >= min(64, b.r - pr.col0)) return;
    cplx<A> s = {A(0), A(0)};
    for (int q = 0; q < pr.nslots; ++q) s = s + tpart[(int64_t)(pr.slot0 + q) * kWave + lane];
    t[b.toff + pr.col0 + lane] = s;
}

// acc[k] += sum_j col_j[row_k] * w_j over `ncol` columns of a column-major
// panel starting at `base` with leading dimension ld; w_j read from `wv`.
template <typename S, typename A, int RPL>
__device__ inline void panel_accum(cplx<A> (&acc)[RPL], const cplx<S> *__restrict__ base,
                                   int64_t ld, const cplx<A> *__restrict__ wv, int32_t ncol,
                                   int32_t r0, int32_t rows, int lane) {
    int32_t j = 0;
    for (; j + 8 <= ncol; j += 8) {
        cplx<A> w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = wv[j + u];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int32_t row = r0 + lane + k * kWave;
            if (row < rows) {
                cplx<S> c[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) c[u] = ld_stream(base + (j + u) * ld + row);
#pragma unroll
                for (int u = 0; u < 8; ++u) fma_(acc[k], cvt<A>(c[u]), w[u]);
            }
        }
    }
    for (; j < ncol; ++j) {
        const cplx<A> w = wv[j];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int32_t row = r0 + lane + k * kWave;
            if (row < rows) fma_(acc[k], cvt<A>(ld_stream(base + j * ld + row)), w);
        }
    }
}

// Complex64 variant: each lane owns row pairs (2q, 2q+1) and reads both with
// one 16-byte load; panels start on even rows and have even leading
// dimensions (padded layout), so every load is aligned.  When a leaf has at
// most 32 row pairs (RPL = 1), the wave splits into G = 64 / npairs groups of
// npairs lanes and group g takes the columns g, g + G, ...: every load
// instruction then moves about a full wave's worth of bytes.
template <int RPL>
__device__ inline void panel_accum_pair(cplx<float> (&acc)[2 * RPL],
                                        const cplx<float> *__restrict__ base, int64_t ld,
                                        const cplx<float> *__restrict__ wv, int32_t ncol,
                                        int32_t p0, int32_t npairs, int lane) {
    const float4 *b4 = reinterpret_cast<const float4 *>(base);
    const int64_t ld4 = ld >> 1;
    if (RPL == 1 && npairs <= kWave / 2) {
        const int G = kWave / npairs, g = lane / npairs, q = lane - g * npairs;
        if (g >= G) return;
        int32_t j = g;
        for (; j + 7 * G < ncol; j += 8 * G) {
            cplx<float> w[8];
            float4 c[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                w[u] = wv[j + u * G];
                c[u] = ld_stream(b4 + (int64_t)(j + u * G) * ld4 + q);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                fma_(acc[0], cplx<float>{c[u].x, c[u].y}, w[u]);
                fma_(acc[1], cplx<float>{c[u].z, c[u].w}, w[u]);
            }
        }
        for (; j < ncol; j += G) {
            const cplx<float> w = wv[j];
            const float4 c = ld_stream(b4 + (int64_t)j * ld4 + q);
            fma_(acc[0], cplx<float>{c.x, c.y}, w);
            fma_(acc[1], cplx<float>{c.z, c.w}, w);
        }
        return;
    }
    int32_t j = 0;
    for (; j + 8 <= ncol; j += 8) {
        cplx<float> w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = wv[j + u];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int32_t q = p0 + lane + k * kWave;
            if (q < npairs) {
                float4 c[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) c[u] = ld_stream(b4 + (j + u) * ld4 + q);
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    fma_(acc[2 * k], cplx<float>{c[u].x, c[u].y}, w[u]);
                    fma_(acc[2 * k + 1], cplx<float>{c[u].z, c[u].w}, w[u]);
                }
            }
        }
    }
    for (; j < ncol; ++j) {
        const cplx<float> w = wv[j];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int32_t q = p0 + lane + k * kWave;
            if (q < npairs) {
                const float4 c = ld_stream(b4 + j * ld4 + q);
                fma_(acc[2 * k], cplx<float>{c.x, c.y}, w);
                fma_(acc[2 * k + 1], cplx<float>{c.z, c.w}, w);
            }
        }
    }
}

// OUT = 0: y (type S) = A x; OUT = 1: r (double) = b - A x.
// RPL rows (row pairs for complex64 storage with complex64 accumulation) per
// lane per chunk, NW waves per leaf (autotuned: 4, 8 or 16).
template <typename S, typename A, int OUT, int RPL, int NW>
__global__ void __launch_bounds__(64 * NW) accum_kernel(
    const LeafRow *__restrict__ leaves, const Task *__restrict__ tasks,
    const DenseBlk *__restrict__ dblk, const LowRankBlk *__restrict__ lblk,
    const cplx<S> *__restrict__ dense, const cplx<S> *__restrict__ fac,
    const cplx<A> *__restrict__ xc, const cplx<A> *__restrict__ t,
    const int32_t *__restrict__ perm, void *__restrict__ yout, int64_t ldy, int32_t col,
    const double *__restrict__ bvec) {
    constexpr bool PAIR = sizeof(S) == 4 && sizeof(A) == 4;
    constexpr int RPC = PAIR ? 2 : 1;   // rows per accumulator slot group
    __shared__ cplx<A> red[NW][kWave * RPL * RPC];
    const LeafRow L = leaves[blockIdx.x];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nw = blockDim.x / kWave;
    const int32_t rows = 3 * L.m;
    constexpr int32_t chunk = kWave * RPL * RPC;
    for (int32_t r0 = 0; r0 < rows; r0 += chunk) {
        cplx<A> acc[RPL * RPC];
#pragma unroll
        for (int k = 0; k < RPL * RPC; ++k) acc[k] = {A(0), A(0)};
        for (int32_t ti = L.tbeg + wave; ti < L.tend; ti += nw) {
            const Task tk = tasks[ti];
            const cplx<S> *base;
            int64_t ld;
            const cplx<A> *wv;
            int32_t ncol;
            if (tk.kind == 0) {
                const DenseBlk d = dblk[tk.idx];
                base = dense + d.off + tk.rowoff;
                ld = d.ld;
                wv = xc + 3 * (int64_t)d.cb;
                ncol = 3 * d.n;
            } else {
                const LowRankBlk b = lblk[tk.idx];
                base = fac + b.uoff + tk.rowoff;
                ld = b.ldu;
                wv = t + b.toff;
                ncol = b.r;
            }
            if constexpr (PAIR) {
                panel_accum_pair<RPL>(acc, reinterpret_cast<const cplx<float> *>(base), ld,
                                      reinterpret_cast<const cplx<float> *>(wv), ncol, r0 / 2,
                                      (rows + 1) / 2, lane);
            } else {
                panel_accum<S, A, RPL>(acc, base, ld, wv, ncol, r0, rows, lane);
            }
        }
        // slot (k, h) holds row r0 + RPC * (lane + 64 k) + h
#pragma unroll
        for (int k = 0; k < RPL; ++k)
#pragma unroll
            for (int h = 0; h < RPC; ++h) red[wave][RPC * (lane + k * kWave) + h] = acc[RPC * k + h];
        __syncthreads();
        // column groups (complex64, at most 32 row pairs): row pair q of group
        // g sits in lane g * npairs + q
        const int32_t npairs = (rows + 1) / 2;
        const int G = (PAIR && RPL == 1 && npairs <= kWave / 2) ? kWave / npairs : 1;
        for (int32_t q = threadIdx.x; q < chunk; q += blockDim.x) {
            const int32_t row = r0 + q;
            if (row < rows) {
                cplx<A> s = {A(0), A(0)};
                for (int w = 0; w < nw; ++w)
                    for (int g = 0; g < G; ++g) s = s + red[w][q + 2 * g * npairs];
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
static void launch_project(const hm_matrix *M, const cplx<A> *xc, cplx<A> *tb, cplx<A> *tp,
                           hipStream_t st) {
    if (M->n_ptasks == 0) return;
    hipLaunchKernelGGL((project_kernel<S, A>), dim3((unsigned)ceil_div(M->n_ptasks, 4)), dim3(256),
                       0, st, M->d_lblk.as<LowRankBlk>(), M->d_ptasks.as<ProjTask>(),
                       M->n_ptasks, M->factors<cplx<S>>(), xc, tb, tp);
    HM_HIP_CHECK(hipGetLastError());
    if (M->n_preduce > 0) {
        hipLaunchKernelGGL((project_reduce_kernel<A>), dim3((unsigned)ceil_div(M->n_preduce, 4)),
                           dim3(256), 0, st, M->d_lblk.as<LowRankBlk>(),
                           M->d_preduce.as<ProjReduce>(), M->n_preduce, tp, tb);
        HM_HIP_CHECK(hipGetLastError());
    }
}

template <typename S, typename A, int OUT, int RPL, int NW>
static void launch_accum_nw(const hm_matrix *M, const cplx<A> *xc, const cplx<A> *tb, void *y,
                            int64_t ldy, int32_t col, const double *b, hipStream_t st) {
    hipLaunchKernelGGL((accum_kernel<S, A, OUT, RPL, NW>), dim3(M->n_leaves), dim3(64 * NW), 0, st,
                       M->d_leaves.as<LeafRow>(), M->d_tasks.as<Task>(),
                       M->d_dblk.as<DenseBlk>(), M->d_lblk.as<LowRankBlk>(),
                       M->dense.as<cplx<S>>(), M->factors<cplx<S>>(), xc, tb,
                       M->perm_x.as<int32_t>(), y, ldy, col, b);
    HM_HIP_CHECK(hipGetLastError());
}

template <typename S, typename A, int OUT, int RPL>
static void launch_accum_rpl(const hm_matrix *M, const cplx<A> *xc, const cplx<A> *tb, void *y,
                             int64_t ldy, int32_t col, const double *b, hipStream_t st) {
    switch (M->acc_waves) {
        case 4: launch_accum_nw<S, A, OUT, RPL, 4>(M, xc, tb, y, ldy, col, b, st); break;
        case 16: launch_accum_nw<S, A, OUT, RPL, 16>(M, xc, tb, y, ldy, col, b, st); break;
        default: launch_accum_nw<S, A, OUT, RPL, 8>(M, xc, tb, y, ldy, col, b, st); break;
    }
}

// Rows per lane chosen so that the largest leaf is covered in one chunk.
template <typename S, typename A, int OUT>
static void launch_accum(const hm_matrix *M, const cplx<A> *xc, const cplx<A> *tb, void *y,
                         int64_t ldy, int32_t col, const double *b, hipStream_t st) {
    const int per_lane = (sizeof(S) == 4 && sizeof(A) == 4) ? 128 : 64;   // rows per RPL unit
    const int rpl =
        (int)std::min<int64_t>(4, std::max<int64_t>(1, ceil_div(3 * M->max_leaf, per_lane)));
    switch (rpl) {
        case 1: launch_accum_rpl<S, A, OUT, 1>(M, xc, tb, y, ldy, col, b, st); break;
        case 2: launch_accum_rpl<S, A, OUT, 2>(M, xc, tb, y, ldy, col, b, st); break;
        case 3: launch_accum_rpl<S, A, OUT, 3>(M, xc, tb, y, ldy, col, b, st); break;
        default: launch_accum_rpl<S, A, OUT, 4>(M, xc, tb, y, ldy, col, b, st); break;
    }
}

// The three launches of one column with explicit workspaces: xc (3 ny
// entries), tb (sum of ranks) and tp (proj_slots x 64 partial sums).
template <typename S, typename A>
static void launch_matvec_col_ws(const hm_matrix *M, const void *x, int64_t ldx, int32_t col,
                                 void *y, int64_t ldy, const double *b, hipStream_t st,
                                 cplx<A> *xc, cplx<A> *tb, cplx<A> *tp) {
    const int64_t ny = M->ny;
    const auto *perm_y = M->p.same ? M->perm_x.as<int32_t>() : M->perm_y.as<int32_t>();
    // The FP64 residual (b != nullptr) takes a complex128 x whatever the storage type.
    if (b == nullptr)
        hipLaunchKernelGGL((gather_kernel<S, A>), dim3(ceil_div(3 * ny, 256)), dim3(256), 0, st,
                           static_cast<const cplx<S> *>(x), ldx, col, perm_y, ny, xc);
    else
        hipLaunchKernelGGL((gather_kernel<double, A>), dim3(ceil_div(3 * ny, 256)), dim3(256), 0,
                           st, static_cast<const cplx<double> *>(x), ldx, col, perm_y, ny, xc);
    HM_HIP_CHECK(hipGetLastError());
    launch_project<S, A>(M, xc, tb, tp, st);
    if (b == nullptr)
        launch_accum<S, A, 0>(M, xc, tb, y, ldy, col, nullptr, st);
    else
        launch_accum<S, A, 1>(M, xc, tb, y, ldy, col, b, st);
}

template <typename S, typename A>
void launch_matvec_col(const hm_matrix *M, const void *x, int64_t ldx, int32_t col, void *y,
                       int64_t ldy, const double *b, hipStream_t st) {
    launch_matvec_col_ws<S, A>(M, x, ldx, col, y, ldy, b, st, M->ws_xc.as<cplx<A>>(),
                               M->ws_t.as<cplx<A>>(), M->tpart.as<cplx<A>>());
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
    launch_project<S, A>(M, xc, tb, M->tpart.as<cplx<A>>(), st);
    HM_HIP_CHECK(hipEventRecord(ev[2], st));
    launch_accum<S, A, 0>(M, xc, tb, y, 1, 0, nullptr, st);
    HM_HIP_CHECK(hipEventRecord(ev[3], st));
    HM_HIP_CHECK(hipEventSynchronize(ev[3]));
    for (int k = 0; k < 3; ++k) {
        float tms = 0;
        HM_HIP_CHECK(hipEventElapsedTime(&tms, ev[k], ev[k + 1]));
        ms3[k] += tms;
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

// ---- allocation-free product -------------------------------------------------
// The workspaces of hm_matvec_noalloc live in one fixed device array per GPU.
// In host code `scratch` names a host-side stand-in, not device memory: only
// the address from hipGetSymbolAddress (kept per device below) reaches kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_dev[64] = {};

// Device address of this GPU's `scratch`, looked up once per device with the
// device current.
unsigned char *scratch_address() {
    int dev = 0;
    HM_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) throw StatusError(HM_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HM_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw StatusError(HM_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch");
        g_scratch_dev[dev] = p;
    }
    return static_cast<unsigned char *>(g_scratch_dev[dev]);
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

template <typename S>
void matvec_noalloc_cols(const hm_matrix *M, const void *x, void *y, int32_t nrhs,
                         hipStream_t st) {
    using A = S;
    const size_t sa = sizeof(cplx<A>);
    const size_t bx = align256(3 * (size_t)M->ny * sa);
    const size_t bt = align256((size_t)std::max<int64_t>(M->t_len, 1) * sa);
    const size_t bp = align256((size_t)std::max(M->proj_slots, 1) * kWave * sa);
    if (bx + bt + bp > kScratchBytes)
        throw StatusError(HM_ERR_ARG, "hm_matvec_noalloc needs " + std::to_string(bx + bt + bp) +
                                          " bytes of scratch, more than its fixed " +
                                          std::to_string(kScratchBytes));
    unsigned char *base = scratch_address();
    auto *xc = reinterpret_cast<cplx<A> *>(base);
    auto *tb = reinterpret_cast<cplx<A> *>(base + bx);
    auto *tp = reinterpret_cast<cplx<A> *>(base + bx + bt);
    for (int32_t c = 0; c < nrhs; ++c)
        launch_matvec_col_ws<S, A>(M, x, nrhs, c, y, nrhs, nullptr, st, xc, tb, tp);
}
}  // namespace

}  // namespace hm

using namespace hm;

extern "C" hm_status hm_matvec_noalloc(const hm_matrix *A, const void *x, void *y, int32_t nrhs,
                                       void *stream) {
    HM_API_BEGIN
    if (!A || !x || !y) throw StatusError(HM_ERR_ARG, "NULL argument");
    if (nrhs < 1) throw StatusError(HM_ERR_ARG, "nrhs must be >= 1");
    if (A->plan_only) throw StatusError(HM_ERR_STATE, "matrix was built with plan_only");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (A->p.prec == HM_C64)
        matvec_noalloc_cols<float>(A, x, y, nrhs, st);
    else
        matvec_noalloc_cols<double>(A, x, y, nrhs, st);
    return HM_OK;
    HM_API_END
}
