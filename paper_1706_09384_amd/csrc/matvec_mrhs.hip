// Multi-RHS H-matrix product Y = A X (Section 3.1) for complex64 storage,
// on panels of up to 64 right-hand sides with FP32 matrix cores.
//
// Each block product is a small complex GEMM: a dense tile times X_sigma, and
// for a low-rank block T = V^* X_sigma followed by U T.  A complex product
// C += A B takes three real ones (Gauss):
//   P1 += Re A Re B,  P2 += Im A Im B,  P3 += (Re A + Im A)(Re B + Im B),
//   Re C = P1 - P2,   Im C = P3 - P1 - P2,
// each issued as v_mfma_f32_16x16x4_f32 steps: 16 output rows x 16 columns,
// 4 values of the contraction index per step.  One wave owns 16 output rows
// and all 64 columns (4 column blocks x 3 products = 12 accumulator tiles).
//
// Operand layout of one 16x16x4 step (CDNA): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; the 4 accumulator values of lane l are the rows
// 4 (l / 16) + v, v = 0..3, of column l % 16.  With column-major A panels,
// lanes 0..15 read 16 consecutive complex entries of one column (128 bytes),
// and with row-major X / T, lanes 0..15 read 16 consecutive right-hand sides.
//
// Passes (no atomics; every output row is written by one wave):
//   gather   X (original order, columns col0..col0+ncols) -> X64 (cluster
//            order, 64 columns, zero beyond ncols)
//   project  T_b = V_b^* X64[sigma_b]: one wave per (block, 16 rows of T,
//            chunk of the contraction), partial chunks summed by a reduction
//            pass in fixed order
//   accum    one wave per (leaf row cluster, 16 of its rows): the sum over
//            the leaf's dense tiles and low-rank U rows, scattered to the
//            original order.
#include <algorithm>

#include "internal.hpp"

namespace hm {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline v4f mfma16(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// acc[cb], acc[4 + cb], acc[8 + cb]: P1, P2, P3 of column block cb.
__device__ inline void mr_step(v4f (&acc)[12], float ar, float ai, const float2 (&x)[4]) {
    const float as = ar + ai;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        acc[cb] = mfma16(ar, x[cb].x, acc[cb]);
        acc[4 + cb] = mfma16(ai, x[cb].y, acc[4 + cb]);
        acc[8 + cb] = mfma16(as, x[cb].x + x[cb].y, acc[8 + cb]);
    }
}

// Entry (v, cb) of the product from the three accumulators.
__device__ inline float2 mr_out(const v4f (&acc)[12], int cb, int v) {
    const float p1 = acc[cb][v], p2 = acc[4 + cb][v];
    return make_float2(p1 - p2, acc[8 + cb][v] - p1 - p2);
}

// acc += op(A)[rows, 0..K) * B[0..K, 0..64): A element (i, k) at a[k * ld + i]
// (conjugated when CONJ), valid for lanes with iv; B row-major with 64
// complex columns.  Loads of the next step are issued before the current
// step's matrix instructions.
template <bool CONJ>
__device__ inline void mr_panel(v4f (&acc)[12], const float2 *__restrict__ a, int64_t ld, int i,
                                bool iv, const float2 *__restrict__ b, int32_t K, int lane) {
    const int kq = lane >> 4, cl = lane & 15;
    const float2 zero = make_float2(0.f, 0.f);
    float2 av = zero, xv[4] = {zero, zero, zero, zero};
    {
        const int32_t kk = kq;
        if (kk < K) {
            if (iv) av = a[(int64_t)kk * ld + i];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) xv[cb] = b[(int64_t)kk * 64 + 16 * cb + cl];
        }
    }
    for (int32_t k = 0; k < K; k += 4) {
        float2 an = zero, xn[4] = {zero, zero, zero, zero};
        const int32_t kk = k + 4 + kq;
        if (kk < K) {
            if (iv) an = a[(int64_t)kk * ld + i];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) xn[cb] = b[(int64_t)kk * 64 + 16 * cb + cl];
        }
        mr_step(acc, av.x, CONJ ? -av.y : av.y, xv);
        av = an;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) xv[cb] = xn[cb];
    }
}

__global__ void __launch_bounds__(256) mr_gather_kernel(const float2 *__restrict__ x, int64_t ldx,
                                                        int32_t col0, int32_t ncols,
                                                        const int32_t *__restrict__ perm,
                                                        int64_t npts, float2 *__restrict__ x64) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 3 * npts * 64) return;
    const int64_t row = q >> 6;
    const int c = (int)(q & 63);
    const int64_t p = row / 3, a = row - 3 * p;
    x64[q] = c < ncols ? x[(3 * (int64_t)perm[p] + a) * ldx + col0 + c] : make_float2(0.f, 0.f);
}

__global__ void __launch_bounds__(256) mr_project_kernel(const MrProjItem *__restrict__ items,
                                                         int32_t nitems,
                                                         const LowRankBlk *__restrict__ lblk,
                                                         const float2 *__restrict__ fac,
                                                         const float2 *__restrict__ x64,
                                                         float2 *__restrict__ t64,
                                                         float2 *__restrict__ tpart) {
    const int lane = threadIdx.x & 63;
    const int32_t w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nitems) return;   // whole waves only; no barriers below
    const MrProjItem it = items[w];
    const LowRankBlk b = lblk[it.blk];
    v4f acc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
    // A(i, k) = conj(V(k0 + k, j0 + i)); V row-major with row stride ldv
    const int j = it.j0 + (lane & 15);
    mr_panel<true>(acc, fac + b.voff + (int64_t)it.k0 * b.ldv + it.j0, b.ldv, lane & 15, j < b.r,
                   x64 + (3 * (int64_t)b.cb + it.k0) * 64, it.klen, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = 4 * (lane >> 4) + v;
        if (it.j0 + row >= b.r) continue;
        float2 *dst = it.slot < 0 ? t64 + ((int64_t)b.toff + it.j0 + row) * 64
                                  : tpart + ((int64_t)it.slot * 16 + row) * 64;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
            dst[16 * cb + (lane & 15)] = mr_out(acc, cb, v);
    }
}

// T rows j0..j0+15 of a block = sum of its chunk partials, in chunk order.
__global__ void __launch_bounds__(256) mr_project_reduce_kernel(
    const MrProjReduce *__restrict__ red, const LowRankBlk *__restrict__ lblk,
    const float2 *__restrict__ tpart, float2 *__restrict__ t64) {
    const MrProjReduce pr = red[blockIdx.x];
    const LowRankBlk b = lblk[pr.blk];
    for (int e = threadIdx.x; e < 16 * 64; e += blockDim.x) {
        const int row = e >> 6;
        if (pr.j0 + row >= b.r) continue;
        float2 s = make_float2(0.f, 0.f);
        for (int q = 0; q < pr.nslots; ++q) {
            const float2 v = tpart[(int64_t)(pr.slot0 + q) * 16 * 64 + e];
            s.x += v.x;
            s.y += v.y;
        }
        t64[((int64_t)b.toff + pr.j0 + row) * 64 + (e & 63)] = s;
    }
}

__global__ void __launch_bounds__(256) mr_accum_kernel(
    const MrAccItem *__restrict__ items, int32_t nitems, const LeafRow *__restrict__ leaves,
    const Task *__restrict__ tasks, const DenseBlk *__restrict__ dblk,
    const LowRankBlk *__restrict__ lblk, const float2 *__restrict__ dense,
    const float2 *__restrict__ fac, const float2 *__restrict__ x64,
    const float2 *__restrict__ t64, const int32_t *__restrict__ perm, float2 *__restrict__ y,
    int64_t ldy, int32_t col0, int32_t ncols) {
    const int lane = threadIdx.x & 63;
    const int32_t w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nitems) return;   // whole waves only; no barriers below
    const MrAccItem it = items[w];
    const LeafRow L = leaves[it.leaf];
    const int32_t rows = 3 * L.m;
    const int i = it.row0 + (lane & 15);
    const bool iv = i < rows;
    v4f acc[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int32_t ti = L.tbeg; ti < L.tend; ++ti) {
        const Task tk = tasks[ti];
        if (tk.kind == 0) {
            const DenseBlk d = dblk[tk.idx];
            mr_panel<false>(acc, dense + d.off + tk.rowoff, d.ld, i, iv,
                            x64 + 3 * (int64_t)d.cb * 64, 3 * d.n, lane);
        } else {
            const LowRankBlk b = lblk[tk.idx];
            mr_panel<false>(acc, fac + b.uoff + tk.rowoff, b.ldu, i, iv,
                            t64 + (int64_t)b.toff * 64, b.r, lane);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int32_t row = it.row0 + 4 * (lane >> 4) + v;
        if (row >= rows) continue;
        const int32_t p = row / 3, a = row - 3 * p;
        float2 *dst = y + (3 * (int64_t)perm[L.rb + p] + a) * ldy + col0;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int c = 16 * cb + (lane & 15);
            if (c < ncols) dst[c] = mr_out(acc, cb, v);
        }
    }
}

}  // namespace

void ensure_mrhs_workspace(const hm_matrix *M) {
    if (M->ws_x64.p) return;
    M->ws_x64.alloc(3 * std::max<int64_t>(M->ny, 1) * 64 * sizeof(float2));
    M->ws_t64.alloc(std::max<int64_t>(M->t_len, 1) * 64 * sizeof(float2));
    M->ws_tp64.alloc(std::max<int64_t>(M->mr_nslots, 1) * 16 * 64 * sizeof(float2));
}

// Launches of one panel; when ev is non-null, events ev[0..3] bracket the
// gather, project and accum passes.
void launch_matvec_mrhs(const hm_matrix *M, const void *x, int64_t ldx, int32_t col0,
                        int32_t ncols, void *y, int64_t ldy, hipStream_t st, hipEvent_t *ev) {
    ensure_mrhs_workspace(M);
    const auto *perm_y = M->p.same ? M->perm_x.as<int32_t>() : M->perm_y.as<int32_t>();
    auto *x64 = M->ws_x64.as<float2>();
    auto *t64 = M->ws_t64.as<float2>();
    auto *tp = M->ws_tp64.as<float2>();
    const auto *fac = M->factors<float2>();
    if (ev) HM_HIP_CHECK(hipEventRecord(ev[0], st));
    hipLaunchKernelGGL(mr_gather_kernel, dim3((unsigned)ceil_div(3 * M->ny * 64, 256)), dim3(256), 0,
                       st, static_cast<const float2 *>(x), ldx, col0, ncols, perm_y, M->ny, x64);
    HM_HIP_CHECK(hipGetLastError());
    if (ev) HM_HIP_CHECK(hipEventRecord(ev[1], st));
    if (M->n_mrproj > 0) {
        hipLaunchKernelGGL(mr_project_kernel, dim3((unsigned)ceil_div(M->n_mrproj, 4)), dim3(256),
                           0, st, M->d_mrproj.as<MrProjItem>(), M->n_mrproj,
                           M->d_lblk.as<LowRankBlk>(), fac, x64, t64, tp);
        HM_HIP_CHECK(hipGetLastError());
    }
    if (M->n_mrred > 0) {
        hipLaunchKernelGGL(mr_project_reduce_kernel, dim3((unsigned)M->n_mrred), dim3(256), 0, st,
                           M->d_mrred.as<MrProjReduce>(), M->d_lblk.as<LowRankBlk>(), tp, t64);
        HM_HIP_CHECK(hipGetLastError());
    }
    if (ev) HM_HIP_CHECK(hipEventRecord(ev[2], st));
    hipLaunchKernelGGL(mr_accum_kernel, dim3((unsigned)ceil_div(M->n_mracc, 4)), dim3(256), 0, st,
                       M->d_mracc.as<MrAccItem>(), M->n_mracc, M->d_leaves.as<LeafRow>(),
                       M->d_tasks.as<Task>(), M->d_dblk.as<DenseBlk>(),
                       M->d_lblk.as<LowRankBlk>(), M->dense.as<float2>(), fac, x64, t64,
                       M->perm_x.as<int32_t>(), static_cast<float2 *>(y), ldy, col0, ncols);
    HM_HIP_CHECK(hipGetLastError());
    if (ev) HM_HIP_CHECK(hipEventRecord(ev[3], st));
}

}  // namespace hm
