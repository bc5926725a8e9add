// Recompression of ACA factors (Section 3.2): B = U V^* = Q_U R_U R_V^* Q_V^*,
// truncated SVD of the small r x r core R_U R_V^* = P S L^*, then
// U' = Q_U P S^1/2 and V' = Q_V L S^1/2 keeping the leading singular values.
//
// GPU form (all FP64, whatever the storage precision; the products run on
// the FP64 matrix cores):
//   gram     G_U = U^* U and G_V = V^* V, 32x32 output tiles per workgroup,
//            one wave per 16x16 quarter;
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
#include <algorithm>
#include <climits>
#include <mutex>

#include "internal.hpp"
#include "mfma_gemm.hpp"

namespace hm {

// Per-block FP64 work area (complex doubles): r x r column-major slots
// 0 R_U (from G_U), 1 R_V (from G_V), 2 M (then M J), 3 J or the unrotated
// core, 4 W_U, 5 W_V, 6 right singular vectors L (r x keep), 7 (last, with
// r^2 + 2r complex doubles: enough for 3r doubles and r ints for every
// r >= 1) column scales, singular values and their ranking.
__host__ __device__ inline int64_t rc_slot(int32_t r, int s) { return (int64_t)s * r * r; }

struct GramItem {
    int32_t blk, which, ta, tc;   // which 0 = U, 1 = V; ta <= tc tile indices
};

constexpr int kGT = 64;   // output tile: 64 x 64 per workgroup, 32 x 32 per wave
constexpr int kGS = 16;   // rows of X staged in LDS per contraction slab

// G_X = X^* X on the FP64 matrix cores (v_mfma_f64_16x16x4f64: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16], and accumulator element e is
// C[4e + l / 16][l % 16]).  One workgroup per 64 x 64 output tile (upper
// triangle of tiles); the four waves take its 32 x 32 quadrants, and a wave
// skips the 16 x 16 sub-tiles that lie outside the matrix or wholly below the
// diagonal.  The contraction runs over slabs of 16 rows of the two 64-column
// panels, staged in LDS and converted to FP64 once, so that every factor entry
// is read from memory once per tile instead of once per wave; the next slab
// is loaded into registers while the current one is multiplied.
// Re G = Xr^T Xr + Xi^T Xi and Im G = Xr^T Xi - Xi^T Xr, from three real
// products.
template <typename R>
__global__ void __launch_bounds__(256) gram_mfma_kernel(const RcBlk *__restrict__ blks,
                                                        const GramItem *__restrict__ items,
                                                        const cplx<R> *__restrict__ fac,
                                                        cplx<double> *__restrict__ work) {
    __shared__ cplx<double> sa[kGS][kGT + 1], sc[kGS][kGT + 1];
    const GramItem it = items[blockIdx.x];
    const RcBlk b = blks[it.blk];
    const int r = b.r;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wa = wave & 1, wc = wave >> 1, g = lane >> 4, l16 = lane & 15;
    const int64_t rows = 3 * (int64_t)(it.which == 0 ? b.m : b.n);
    const cplx<R> *X = fac + (it.which == 0 ? b.uoff : b.voff);
    cplx<double> *G = work + b.goff + rc_slot(r, it.which);
    const int a0 = it.ta * kGT, c0 = it.tc * kGT;
    const bool diag = it.ta == it.tc;
    bool act[2][2];
    bool any = false;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int ab = a0 + 32 * wa + 16 * i, cb = c0 + 32 * wc + 16 * j;
            act[i][j] = ab < r && cb < r && ab <= cb + 15;
            any = any || act[i][j];
        }
    // conj(a) b as three real products (Gauss): P1 = Re a Re b,
    // P2 = -Im a Im b, P3 = (Re a - Im a)(Re b + Im b); Re G = P1 - P2,
    // Im G = P3 - P1 - P2
    mf64x4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) p1[i][j] = p2[i][j] = p3[i][j] = mf64x4{0, 0, 0, 0};
    cplx<double>(*scp)[kGT + 1] = diag ? sa : sc;
    // staging: entry tid + 256 s of a slab is (row (tid + 256 s) % 16, column
    // (tid + 256 s) / 16), so that 16 lanes read 16 consecutive rows of a column
    constexpr int kPer = kGS * kGT / 256;
    cplx<R> na[kPer], nc[kPer];
    auto fetch = [&](int64_t q0) {
#pragma unroll
        for (int s = 0; s < kPer; ++s) {
            const int e = tid + 256 * s, col = e / kGS;
            const int64_t q = q0 + e % kGS;
            na[s] = (a0 + col < r && q < rows) ? X[(int64_t)(a0 + col) * rows + q]
                                               : cplx<R>{R(0), R(0)};
            if (!diag)
                nc[s] = (c0 + col < r && q < rows) ? X[(int64_t)(c0 + col) * rows + q]
                                                   : cplx<R>{R(0), R(0)};
        }
    };
    fetch(0);
    for (int64_t q0 = 0; q0 < rows; q0 += kGS) {
#pragma unroll
        for (int s = 0; s < kPer; ++s) {
            const int e = tid + 256 * s, col = e / kGS, row = e % kGS;
            sa[row][col] = cvt<double>(na[s]);
            if (!diag) sc[row][col] = cvt<double>(nc[s]);
        }
        if (q0 + kGS < rows) fetch(q0 + kGS);
        __syncthreads();
        if (any) {
#pragma unroll
            for (int s4 = 0; s4 < kGS; s4 += 4) {
                cplx<double> A[2], B[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    A[t] = sa[s4 + g][32 * wa + 16 * t + l16];
                    B[t] = scp[s4 + g][32 * wc + 16 * t + l16];
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        if (act[i][j]) {
                            p1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[i].re, B[j].re,
                                                                            p1[i][j], 0, 0, 0);
                            p2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-A[i].im, B[j].im,
                                                                            p2[i][j], 0, 0, 0);
                            p3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                A[i].re - A[i].im, B[j].re + B[j].im, p3[i][j], 0, 0, 0);
                        }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            if (act[i][j])
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int a = a0 + 32 * wa + 16 * i + 4 * e + g;
                    const int c = c0 + 32 * wc + 16 * j + l16;
                    if (a < r && c < r && a <= c) {
                        const double gr = p1[i][j][e] - p2[i][j][e];
                        const double gi = a == c ? 0.0 : p3[i][j][e] - p1[i][j][e] - p2[i][j][e];
                        G[a + (int64_t)c * r] = {gr, gi};
                        G[c + (int64_t)a * r] = {gr, -gi};
                    }
                }
}

__device__ inline double wave_sumd(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// In-place upper Cholesky G = R^* R of an r x r Hermitian PSD matrix with
// unit diagonal (column-major); entries below the diagonal are zeroed.
// A pivot <= tol marks a numerically dependent column: its row of R is zero.
__device__ void chol_upper(cplx<double> *G, int r, double tol, double *sh) {
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    for (int k = 0; k < r; ++k) {
        if (wave == 0) {
            double d = 0;
            for (int i = lane; i < k; i += 64) d += abs2(G[i + (int64_t)k * r]);
            d = wave_sumd(d);
            if (lane == 0) {
                d = G[k + (int64_t)k * r].re - d;
                const double rk = d > tol ? sqrt(d) : 0.0;
                G[k + (int64_t)k * r] = {rk, 0.0};
                sh[0] = rk;
            }
        }
        __syncthreads();
        const double rk = sh[0];
        const cplx<double> *rkcol = G + (int64_t)k * r;
        for (int j = k + 1 + tid; j < r; j += blockDim.x) {
            cplx<double> *cj = G + (int64_t)j * r;
            cplx<double> s = cj[k];
            for (int i = 0; i < k; ++i) s = s - cmul(rkcol[i], cj[i]);
            cj[k] = rk > 0.0 ? (1.0 / rk) * s : cplx<double>{0, 0};
        }
        __syncthreads();
    }
    for (int64_t q = tid; q < (int64_t)r * r; q += blockDim.x) {
        const int i = (int)(q % r), j = (int)(q / r);
        if (i > j) G[q] = {0, 0};
    }
    __syncthreads();
}

// The same factorisation for a matrix in global memory (ranks whose r x r
// matrices do not fit in LDS): each off-diagonal entry R(k, j) is one wave's
// 64-lane dot product over i < k instead of one thread's serial loop, so the
// k-th step costs a few load latencies rather than k of them.
__device__ void chol_upper_wide(cplx<double> *G, int r, double tol, double *sh) {
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int nw = blockDim.x / 64;
    for (int k = 0; k < r; ++k) {
        if (wave == 0) {
            double d = 0;
            for (int i = lane; i < k; i += 64) d += abs2(G[i + (int64_t)k * r]);
            d = wave_sumd(d);
            if (lane == 0) {
                d = G[k + (int64_t)k * r].re - d;
                const double rk = d > tol ? sqrt(d) : 0.0;
                G[k + (int64_t)k * r] = {rk, 0.0};
                sh[0] = rk;
            }
        }
        __syncthreads();
        const double rk = sh[0];
        const cplx<double> *rkcol = G + (int64_t)k * r;
        for (int j = k + 1 + wave; j < r; j += nw) {
            cplx<double> *cj = G + (int64_t)j * r;
            double sr = 0, si = 0;
            for (int i = lane; i < k; i += 64) {
                const cplx<double> t = cmul(rkcol[i], cj[i]);
                sr += t.re;
                si += t.im;
            }
            sr = wave_sumd(sr);
            si = wave_sumd(si);
            if (lane == 0) {
                const cplx<double> s = cj[k] - cplx<double>{sr, si};
                cj[k] = rk > 0.0 ? (1.0 / rk) * s : cplx<double>{0, 0};
            }
        }
        __syncthreads();
    }
    for (int64_t q = tid; q < (int64_t)r * r; q += blockDim.x) {
        const int i = (int)(q % r), j = (int)(q / r);
        if (i > j) G[q] = {0, 0};
    }
    __syncthreads();
}

// One rotation of the one-sided Jacobi method on columns x, y (length r, LDS)
// with the matching columns jx, jy of J, executed by a group of gs lanes
// (gs a power of two dividing 64; gl = lane index inside the group).
// Returns true if a rotation was applied.
template <bool WITHJ>
__device__ inline bool jacobi_pair(cplx<double> *x, cplx<double> *y, cplx<double> *jx,
                                   cplx<double> *jy, int r, double tol, double tiny, int gl,
                                   int gs) {
    double al = 0, be = 0, gr = 0, gi = 0;
    for (int i = gl; i < r; i += gs) {
        const cplx<double> a = x[i], b = y[i];
        al += abs2(a);
        be += abs2(b);
        gr += a.re * b.re + a.im * b.im;
        gi += a.re * b.im - a.im * b.re;
    }
    for (int o = gs / 2; o > 0; o >>= 1) {
        al += __shfl_xor(al, o, gs);
        be += __shfl_xor(be, o, gs);
        gr += __shfl_xor(gr, o, gs);
        gi += __shfl_xor(gi, o, gs);
    }
    // A column whose squared norm is at the rounding level of the whole
    // matrix (tiny) is numerically zero: its orthogonality is noise, and
    // rotating it would only keep the sweeps from terminating.
    if (al <= tiny || be <= tiny) return false;
    const double ag = sqrt(gr * gr + gi * gi);
    if (!(ag > tol * sqrt(al * be))) return false;
    // Unitary [[c, s], [-s e^{-i phi}, c e^{-i phi}]] diagonalising the 2x2 Gram.
    const double tau = (be - al) / (2.0 * ag);
    const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
    const cplx<double> ph = {gr / ag, -gi / ag};
    const cplx<double> v10 = (-s) * ph, v11 = c * ph;
    for (int i = gl; i < r; i += gs) {
        const cplx<double> a = x[i], b = y[i];
        x[i] = c * a + b * v10;
        y[i] = s * a + b * v11;
        if constexpr (WITHJ) {
            const cplx<double> ja = jx[i], jb = jy[i];
            jx[i] = c * ja + jb * v10;
            jy[i] = s * ja + jb * v11;
        }
    }
    return true;
}

// Position -> column of the round-robin tournament over `n` (even) slots.
__device__ inline int rr_slot(int pos, int round, int n) {
    return pos == 0 ? 0 : 1 + (pos - 1 + round) % (n - 1);
}

// One sweep over all column pairs of the `nc` columns held in LDS at
// lds (column-major, leading dimension r) with the matching columns of J at
// ldj; the pairs of one round are disjoint and run concurrently, each on a
// group of gs lanes sized so that a round fills the workgroup.  Returns
// whether anything rotated.
template <bool WITHJ>
__device__ bool lds_sweep(cplx<double> *lds, cplx<double> *ldj, int nc, int r, double tol,
                          double tiny, int *sh_flag) {
    const int ne = (nc + 1) & ~1;
    const int npairs = ne / 2;
    int gs = 64;
    while (gs > 1 && npairs * gs > (int)blockDim.x) gs >>= 1;
    const int ngroups = blockDim.x / gs;
    const int grp = threadIdx.x / gs, gl = threadIdx.x % gs;
    if (threadIdx.x == 0) *sh_flag = 0;
    __syncthreads();
    bool any = false;
    for (int round = 0; round < ne - 1; ++round) {
        for (int pr = grp; pr < npairs; pr += ngroups) {
            int p = rr_slot(pr, round, ne), q = rr_slot(ne - 1 - pr, round, ne);
            if (p >= nc || q >= nc) continue;
            if (p > q) {
                const int tq = p;
                p = q;
                q = tq;
            }
            any |= jacobi_pair<WITHJ>(lds + (int64_t)p * r, lds + (int64_t)q * r,
                                      WITHJ ? ldj + (int64_t)p * r : nullptr,
                                      WITHJ ? ldj + (int64_t)q * r : nullptr, r, tol, tiny, gl,
                                      gs);
        }
        __syncthreads();
    }
    if (any && gl == 0) *sh_flag = 1;
    __syncthreads();
    const bool res = *sh_flag != 0;
    // every thread has read the flag before anyone may reset it again
    __syncthreads();
    return res;
}

// Squared column norm below which a column of the r x r matrix M counts as
// numerically zero: r u^2 |M|_F^2 (|M|_F is invariant under the rotations).
// Block-wide; every thread returns the value.
__device__ double jacobi_tiny(const cplx<double> *M, int r) {
    __shared__ double sh_nrm[16];
    const int tid = threadIdx.x;
    double v = 0;
    for (int64_t q = tid; q < (int64_t)r * r; q += blockDim.x) v += abs2(M[q]);
    v = wave_sumd(v);
    if (tid % 64 == 0) sh_nrm[tid / 64] = v;
    __syncthreads();
    if (tid == 0) {
        double t = 0;
        for (int w = 0; w < (int)blockDim.x / 64; ++w) t += sh_nrm[w];
        sh_nrm[0] = t;
    }
    __syncthreads();
    const double tiny = r * (2.3e-16 * 2.3e-16) * sh_nrm[0];
    __syncthreads();   // sh_nrm is read before any later reuse
    return tiny;
}

// Columns per LDS block of the block Jacobi method (two blocks, with J when
// the rotations are accumulated, fill lds_elems complex doubles).
__host__ __device__ inline int jacobi_bw(int r, int64_t lds_elems, int nj) {
    const int64_t w = lds_elems / (2 * nj * (int64_t)r);
    return (int)(w > 1 ? w : 1);
}

// One-sided Jacobi SVD of the r x r column-major matrix M (global), in place:
// on exit the columns of M J are mutually orthogonal, M J = P S.  With WITHJ
// the rotations are also applied to J (global, identity on entry), giving
// J = L.  Columns are processed in LDS (with J side by side), the whole
// matrix at once when it fits, else as pairs of column blocks of width bw
// (block Jacobi, round-robin over the blocks).
template <bool WITHJ>
__device__ void jacobi_svd(cplx<double> *M, cplx<double> *J, int r, cplx<double> *lds,
                           int64_t lds_elems, int *sh_flag) {
    const double tol = fmax(1e-14, 4.0 * r * 1.1e-16);
    const int tid = threadIdx.x;
    constexpr int NJ = WITHJ ? 2 : 1;
    const double tiny = jacobi_tiny(M, r);
    if (NJ * (int64_t)r * r <= lds_elems) {
        cplx<double> *ldj = lds + (int64_t)r * r;
        for (int64_t q = tid; q < (int64_t)r * r; q += blockDim.x) {
            lds[q] = M[q];
            if constexpr (WITHJ) ldj[q] = J[q];
        }
        __syncthreads();
        for (int sweep = 0; sweep < 30; ++sweep)
            if (!lds_sweep<WITHJ>(lds, ldj, r, r, tol, tiny, sh_flag)) break;
        for (int64_t q = tid; q < (int64_t)r * r; q += blockDim.x) {
            M[q] = lds[q];
            if constexpr (WITHJ) J[q] = ldj[q];
        }
        __syncthreads();
        return;
    }
    const int bw = jacobi_bw(r, lds_elems, NJ);
    const int nb = (r + bw - 1) / bw;
    const int ne = (nb + 1) & ~1;
    cplx<double> *ldj = lds + 2 * (int64_t)bw * r;
    for (int sweep = 0; sweep < 30; ++sweep) {
        bool any = false;
        for (int round = 0; round < ne - 1; ++round) {
            for (int pr = 0; pr < ne / 2; ++pr) {
                const int bi = rr_slot(pr, round, ne), bj = rr_slot(ne - 1 - pr, round, ne);
                if (bi >= nb || bj >= nb) continue;
                const int c0 = bi * bw, n0 = min(bw, r - c0);
                const int c1 = bj * bw, n1 = min(bw, r - c1);
                const int nc = n0 + n1;
                for (int64_t q = tid; q < (int64_t)nc * r; q += blockDim.x) {
                    const int cc = (int)(q / r), i = (int)(q % r);
                    const int col = cc < n0 ? c0 + cc : c1 + (cc - n0);
                    lds[q] = M[(int64_t)col * r + i];
                    if constexpr (WITHJ) ldj[q] = J[(int64_t)col * r + i];
                }
                __syncthreads();
                any |= lds_sweep<WITHJ>(lds, ldj, nc, r, tol, tiny, sh_flag);
                for (int64_t q = tid; q < (int64_t)nc * r; q += blockDim.x) {
                    const int cc = (int)(q / r), i = (int)(q % r);
                    const int col = cc < n0 ? c0 + cc : c1 + (cc - n0);
                    M[(int64_t)col * r + i] = lds[q];
                    if constexpr (WITHJ) J[(int64_t)col * r + i] = ldj[q];
                }
                __syncthreads();
            }
        }
        if (!any) break;
    }
}

// PHASE 0 runs the whole factorisation of a block in one workgroup.  Blocks
// whose core does not fit in LDS split it: PHASE 1 stops once the core M and
// its negligible column norm (tiny[blockIdx.x]) are formed, the block Jacobi
// sweeps then run as one launch per round over all such blocks
// (jacobi_round_kernel), and PHASE 2 continues from the rotated core.
template <typename R, int NT, int PHASE>
__global__ void __launch_bounds__(NT) factor_kernel(const RcBlk *__restrict__ blks,
                                                     const int32_t *__restrict__ order,
                                                     cplx<double> *__restrict__ work,
                                                     int32_t *__restrict__ newrank, double eps,
                                                     int64_t lds_elems, double *__restrict__ tiny) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cplx<double> *lds = reinterpret_cast<cplx<double> *>(smem_raw);
    __shared__ double sh_s[1];
    __shared__ int sh_i[4];
    const int32_t bi = order[blockIdx.x];
    const RcBlk b = blks[bi];
    const int r = b.r;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    if (r == 0) {
        if (tid == 0 && PHASE != 2) newrank[bi] = 0;
        return;
    }
    cplx<double> *W = work + b.goff;
    cplx<double> *RU = W + rc_slot(r, 0), *RV = W + rc_slot(r, 1), *M = W + rc_slot(r, 2),
                 *J = W + rc_slot(r, 3), *WU = W + rc_slot(r, 4), *WV = W + rc_slot(r, 5);
    cplx<double> *Lw = W + rc_slot(r, 6);
    double *du = reinterpret_cast<double *>(W + rc_slot(r, 7));
    double *dv = du + r;
    double *sv = dv + r;
    int *idx = reinterpret_cast<int *>(sv + r);
    // Column equilibration: G~ = D^-1 G D^-1, D = sqrt(diag G).
    if (PHASE != 2) {
    for (int k = tid; k < r; k += NT) {
        const double a = sqrt(fmax(RU[k + (int64_t)k * r].re, 0.0));
        const double c = sqrt(fmax(RV[k + (int64_t)k * r].re, 0.0));
        du[k] = a > 0 ? a : 1.0;
        dv[k] = c > 0 ? c : 1.0;
    }
    __syncthreads();
    for (int64_t q = tid; q < (int64_t)r * r; q += NT) {
        const int i = (int)(q % r), j = (int)(q / r);
        RU[q] = (1.0 / (du[i] * du[j])) * RU[q];
        RV[q] = (1.0 / (dv[i] * dv[j])) * RV[q];
    }
    __syncthreads();
    const double ctol = 4.0 * r * 1.1e-16;
    for (int side = 0; side < 2; ++side) {
        cplx<double> *G = side == 0 ? RU : RV;
        if ((int64_t)r * r <= lds_elems) {
            // factor in LDS (the dot products of the left-looking sweep are
            // then LDS reads instead of dependent global loads)
            for (int64_t q = tid; q < (int64_t)r * r; q += NT) lds[q] = G[q];
            __syncthreads();
            chol_upper(lds, r, ctol, sh_s);
            for (int64_t q = tid; q < (int64_t)r * r; q += NT) G[q] = lds[q];
            __syncthreads();
        } else {
            chol_upper_wide(G, r, ctol, sh_s);
        }
    }
    }
    // core M = R_U D R_V^*, D = du dv (the block is U~ D V~^*), written to dst
    auto form_core = [&](cplx<double> *dst) {
        mfma_gemm(
            r, r, r,
            [&](int i, int k) {
                return (du[k] * dv[k]) * (i <= k ? RU[i + (int64_t)k * r] : cplx<double>{0, 0});
            },
            [&](int k, int j) { return j <= k ? conj(RV[j + (int64_t)k * r]) : cplx<double>{0, 0}; },
            [&](int i, int j, cplx<double> v) { dst[i + (int64_t)j * r] = v; });
    };
    // singular values = column norms of M J, ranked in descending order; keep =
    // smallest k with sum_{i >= k} s_i^2 <= eps^2 sum s_i^2 (Frobenius tail)
    auto rank_and_keep = [&]() -> int {
        for (int c = wave; c < r; c += NT / 64) {
            double s = 0;
            for (int i = lane; i < r; i += 64) s += abs2(M[i + (int64_t)c * r]);
            s = wave_sumd(s);
            if (lane == 0) sv[c] = sqrt(s);
        }
        __syncthreads();
        // a non-finite value ranks last, so that idx is a permutation
        // whatever the input (NaN compares false both ways)
        auto key = [](double x) { return x <= 1.7976931348623157e308 ? x : -1.0; };
        for (int c = tid; c < r; c += NT) {
            const double v = key(sv[c]);
            int pos = 0;
            for (int k = 0; k < r; ++k) {
                const double w = key(sv[k]);
                if (w > v || (w == v && k < c)) ++pos;
            }
            idx[pos] = c;
        }
        __syncthreads();
        if (tid == 0) {
            double tot = 0;
            for (int k = 0; k < r; ++k) tot += sv[idx[k]] * sv[idx[k]];
            int kp = 0;
            if (tot > 0.0) {
                double tail = 0;
                kp = r;
                for (int k = r; k >= 0; --k) {
                    if (tail <= eps * eps * tot)
                        kp = k;
                    else
                        break;
                    if (k > 0) tail += sv[idx[k - 1]] * sv[idx[k - 1]];
                }
            }
            sh_i[1] = kp;
        }
        __syncthreads();
        return sh_i[1];
    };
    // Right singular vectors.  L = M0^* P S^-1 from the unrotated core M0 is
    // cheap, but a left vector P_c that the sweeps left at angle tau (their
    // orthogonality tolerance) to P_1 puts an error of tau s_1 / s_c into
    // L_c, and the product U' V'^* inherits tau s_1^2 / s_c: 3e-10 relative
    // at eps = 1e-4.  That is far below the rounding of complex64 storage,
    // but not of complex128, so complex128 always accumulates the rotations
    // in J (L = J, error of order tau s_c), and complex64 only when a kept
    // singular value is far below s_1.
    constexpr bool kAlwaysJ = sizeof(R) == 8;
    auto identity_J = [&]() {
        for (int64_t q = tid; q < (int64_t)r * r; q += NT)
            J[q] = (q % r == q / r) ? cplx<double>{1, 0} : cplx<double>{0, 0};
        __syncthreads();
    };
    if (PHASE == 1) {
        form_core(M);
        if (kAlwaysJ) identity_J();
        const double t = jacobi_tiny(M, r);
        if (tid == 0) tiny[blockIdx.x] = t;
        return;
    }
    if (PHASE == 0) {
        form_core(M);
        if (kAlwaysJ) {
            identity_J();
            jacobi_svd<true>(M, J, r, lds, lds_elems, &sh_i[0]);
        } else {
            jacobi_svd<false>(M, nullptr, r, lds, lds_elems, &sh_i[0]);
        }
    }
    int keep = rank_and_keep();
    const bool useJ = kAlwaysJ || (keep > 0 && sv[idx[keep - 1]] < 1e-6 * sv[idx[0]]);
    if (useJ && !kAlwaysJ) {
        form_core(M);
        for (int64_t q = tid; q < (int64_t)r * r; q += NT)
            J[q] = (q % r == q / r) ? cplx<double>{1, 0} : cplx<double>{0, 0};
        __syncthreads();
        jacobi_svd<true>(M, J, r, lds, lds_elems, &sh_i[0]);
        keep = rank_and_keep();
    } else if (!useJ) {
        form_core(J);   // J slot holds M0
        // L[:, c] = M0^* (M J)[:, idx_c] / s_c^2
        mfma_gemm(
            r, keep, r, [&](int j, int i) { return conj(J[i + (int64_t)j * r]); },
            [&](int i, int c) { return M[i + (int64_t)idx[c] * r]; },
            [&](int j, int c, cplx<double> v) {
                const double sc = sv[idx[c]];
                Lw[j + (int64_t)c * r] = (1.0 / (sc * sc)) * v;
            });
    }
    // W_U = D_v R_V^* L_r S_r^-1/2,  W_V = D_u R_U^* P_r S_r^-1/2 with
    // P_r = (M J)[:, idx] / s
    mfma_gemm(
        r, keep, r,
        [&](int k, int j) { return j <= k ? conj(RV[j + (int64_t)k * r]) : cplx<double>{0, 0}; },
        [&](int j, int c) { return useJ ? J[j + (int64_t)idx[c] * r] : Lw[j + (int64_t)c * r]; },
        [&](int k, int c, cplx<double> v) {
            WU[k + (int64_t)c * r] = (dv[k] / sqrt(sv[idx[c]])) * v;
        });
    mfma_gemm(
        r, keep, r,
        [&](int k, int i) { return i <= k ? conj(RU[i + (int64_t)k * r]) : cplx<double>{0, 0}; },
        [&](int i, int c) { return M[i + (int64_t)idx[c] * r]; },
        [&](int k, int c, cplx<double> v) {
            const double sc = sv[idx[c]];
            WV[k + (int64_t)c * r] = (du[k] / (sc * sqrt(sc))) * v;
        });
    if (tid == 0) newrank[bi] = keep;
}

// One round of the block Jacobi sweep of every split block: task t pairs
// the column blocks bi and bj of block order[slot]; the pairs of one round
// are disjoint, so running them side by side gives what the one-workgroup
// sweep computes.  rotated[slot] is set when any pair rotated.
struct JacTask {
    int32_t slot, bi, bj, pad;
};

// WITHJ: the rotations also go to J (slot 3), as in the one-workgroup sweep
// with J (the column blocks are then half as wide).
template <bool WITHJ>
__global__ void __launch_bounds__(1024) jacobi_round_kernel(const RcBlk *__restrict__ blks,
                                                            const int32_t *__restrict__ order,
                                                            const JacTask *__restrict__ tasks,
                                                            cplx<double> *__restrict__ work,
                                                            const double *__restrict__ tiny,
                                                            const int32_t *__restrict__ active,
                                                            int32_t *__restrict__ rotated,
                                                            int64_t lds_elems) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    cplx<double> *lds = reinterpret_cast<cplx<double> *>(smem_raw);
    __shared__ int sh_flag;
    const JacTask t = tasks[blockIdx.x];
    if (!active[t.slot]) return;   // the block converged in an earlier sweep
    const RcBlk b = blks[order[t.slot]];
    const int r = b.r;
    cplx<double> *M = work + b.goff + rc_slot(r, 2);
    cplx<double> *J = work + b.goff + rc_slot(r, 3);
    const double tol = fmax(1e-14, 4.0 * r * 1.1e-16);
    const int bw = jacobi_bw(r, lds_elems, WITHJ ? 2 : 1);
    cplx<double> *ldj = lds + 2 * (int64_t)bw * r;
    const int c0 = t.bi * bw, n0 = min(bw, r - c0);
    const int c1 = t.bj * bw, n1 = min(bw, r - c1);
    const int nc = n0 + n1;
    for (int64_t q = threadIdx.x; q < (int64_t)nc * r; q += blockDim.x) {
        const int cc = (int)(q / r), i = (int)(q % r);
        const int col = cc < n0 ? c0 + cc : c1 + (cc - n0);
        lds[q] = M[(int64_t)col * r + i];
        if constexpr (WITHJ) ldj[q] = J[(int64_t)col * r + i];
    }
    __syncthreads();
    const bool any = lds_sweep<WITHJ>(lds, ldj, nc, r, tol, tiny[t.slot], &sh_flag);
    for (int64_t q = threadIdx.x; q < (int64_t)nc * r; q += blockDim.x) {
        const int cc = (int)(q / r), i = (int)(q % r);
        const int col = cc < n0 ? c0 + cc : c1 + (cc - n0);
        M[(int64_t)col * r + i] = lds[q];
        if constexpr (WITHJ) J[(int64_t)col * r + i] = ldj[q];
    }
    if (any && threadIdx.x == 0) rotated[t.slot] = 1;
}

// Position -> column block of the round-robin tournament (host twin of rr_slot).
inline int rr_slot_host(int pos, int round, int n) {
    return pos == 0 ? 0 : 1 + (pos - 1 + round) % (n - 1);
}

// U' = U W_U (3m x keep), V' = V W_V (3n x keep) into the compact slab, one
// workgroup per (block, factor, 64 rows, 64 output columns).  Wave w owns rows
// 16w .. 16w + 15 of the chunk and every 16-column output tile that holds
// kept columns; its A operand comes straight from the factor (each entry read
// once, the next 16-deep slab loaded into registers while the current one is
// multiplied), and the 16 x 64 slab of W is staged in LDS for the four waves.
// The result is rounded to the storage type.
struct ApplyTask {
    int32_t blk, which, row0, col0;
};

// The product for NT output tiles of 16 columns (NT = 1 .. 4), so that no
// multiply-accumulate sits under a per-tile condition.
template <typename R, int NT>
__device__ void apply_tiles(const RcBlk &b, const ApplyTask &tk, int keep, const cplx<R> *X,
                            const cplx<double> *T, cplx<R> *Y, const int32_t *rowpad,
                            cplx<double> (*sw)[65]) {
    constexpr int kS = 16;
    const int r = b.r;
    const int which = tk.which;
    const int64_t rows = 3 * (int64_t)(which == 0 ? b.m : b.n);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane >> 4, l16 = lane & 15;
    const int col0 = tk.col0;
    const int64_t myrow = (int64_t)tk.row0 + 16 * wave + l16;
    const bool live = (int64_t)tk.row0 + 16 * wave < rows;
    const bool rv = myrow < rows;
    // (Re, Im) of a b as three real products: P1 = Re a Re b, P2 = Im a Im b,
    // P3 = (Re a + Im a)(Re b + Im b); Re = P1 - P2, Im = P3 - P1 - P2
    mf64x4 p1[NT], p2[NT], p3[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) p1[j] = p2[j] = p3[j] = mf64x4{0, 0, 0, 0};
    // next slab: this lane's A entries (row myrow, k = k0 + 4s + g) and its
    // share of the W slab (entry tid + 256 s: k (tid + 256 s) % 16, column
    // (tid + 256 s) / 16)
    cplx<R> nx[4];
    cplx<double> nw[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int k = k0 + 4 * s + g;
            nx[s] = (rv && k < r) ? X[(int64_t)k * rows + myrow] : cplx<R>{R(0), R(0)};
            const int e = tid + 256 * s, col = e / kS, kk = k0 + e % kS;
            nw[s] = (kk < r && col0 + col < keep) ? T[kk + (int64_t)(col0 + col) * r]
                                                  : cplx<double>{0, 0};
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < r; k0 += kS) {
        cplx<double> A[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            A[s] = cvt<double>(nx[s]);
            const int e = tid + 256 * s;
            sw[e % kS][e / kS] = nw[s];
        }
        if (k0 + kS < r) fetch(k0 + kS);
        __syncthreads();
        if (live) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const cplx<double> B = sw[4 * s + g][16 * j + l16];
                    p1[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[s].re, B.re, p1[j], 0, 0, 0);
                    p2[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[s].im, B.im, p2[j], 0, 0, 0);
                    p3[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[s].re + A[s].im, B.re + B.im,
                                                                 p3[j], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    if (!live) return;
    // U' column-major with the padded leaf-segment rows; V' row-major with an
    // even row stride.
    const int64_t ldu = padded_rows(rowpad, b.rb, b.m);
    const int64_t ldv = even_up(keep);
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t row = (int64_t)tk.row0 + 16 * wave + 4 * e + g;
            const int c = col0 + 16 * j + l16;
            if (row < rows && c < keep) {
                const cplx<double> v = {p1[j][e] - p2[j][e], p3[j][e] - p1[j][e] - p2[j][e]};
                const int64_t o = which == 0 ? (int64_t)c * ldu + padded_row(rowpad, b.rb,
                                                                             (int32_t)(row / 3),
                                                                             (int)(row % 3))
                                             : row * ldv + c;
                Y[o] = cvt<R>(v);
            }
        }
}

template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) apply_kernel(const RcBlk *__restrict__ blks,
                                                    const ApplyTask *__restrict__ tasks,
                                                    const cplx<R> *__restrict__ fac,
                                                    const cplx<double> *__restrict__ work,
                                                    const int32_t *__restrict__ newrank,
                                                    const int64_t *__restrict__ outu,
                                                    const int64_t *__restrict__ outv,
                                                    cplx<R> *__restrict__ out,
                                                    const int32_t *__restrict__ rowpad) {
    __shared__ cplx<double> sw[16][65];
    const ApplyTask tk = tasks[blockIdx.x];
    const int bi = tk.blk;
    const RcBlk b = blks[bi];
    const int keep = newrank[bi];
    const cplx<R> *X = fac + (tk.which == 0 ? b.uoff : b.voff);
    const cplx<double> *T = work + b.goff + rc_slot(b.r, tk.which == 0 ? 4 : 5);
    cplx<R> *Y = out + (tk.which == 0 ? outu[bi] : outv[bi]);
    switch (min(4, (keep - tk.col0 + 15) >> 4)) {
    case 1: apply_tiles<R, 1>(b, tk, keep, X, T, Y, rowpad, sw); break;
    case 2: apply_tiles<R, 2>(b, tk, keep, X, T, Y, rowpad, sw); break;
    case 3: apply_tiles<R, 3>(b, tk, keep, X, T, Y, rowpad, sw); break;
    default: apply_tiles<R, 4>(b, tk, keep, X, T, Y, rowpad, sw); break;
    }
}

// Factorisation of the blocks order[q0, q1) whose r x r core exceeds the LDS:
// the core is formed per block (one workgroup each), the block Jacobi sweeps
// run as one launch per tournament round over all of these blocks, with a
// 4-byte-per-block readback after every sweep to retire converged blocks,
// and the truncation and update matrices follow per block.  The sequence of
// rotations applied to each block is the one the one-workgroup sweep applies.
template <typename R>
static void split_jacobi(const std::vector<RcBlk> &blk, const std::vector<int32_t> &order,
                         size_t q0, size_t q1, const RcBlk *d_blk, const int32_t *d_order,
                         double *work, int32_t *d_newrank, double eps, size_t bytes,
                         int64_t lds_elems, hipStream_t st) {
    const int nbig = (int)(q1 - q0);
    auto *W = reinterpret_cast<cplx<double> *>(work);
    DeviceBuf d_tiny, d_active, d_rot, d_tasks;
    d_tiny.alloc(nbig * sizeof(double));
    d_active.alloc(nbig * sizeof(int32_t));
    d_rot.alloc(nbig * sizeof(int32_t));
    // Forming the core needs no dynamic LDS (its Cholesky runs in global
    // memory for these ranks, its products on the matrix cores), so it shares
    // CUs with the other rank classes.
    hipLaunchKernelGGL((factor_kernel<R, 1024, 1>), dim3((unsigned)nbig), dim3(1024), 0, st,
                       d_blk, d_order + q0, W, d_newrank, eps, (int64_t)0, d_tiny.as<double>());
    HM_HIP_CHECK(hipGetLastError());
    // tournament rounds of every block; round t of all blocks in one list
    std::vector<std::vector<JacTask>> rounds;
    for (int s = 0; s < nbig; ++s) {
        const int r = blk[order[q0 + s]].r;
        if (r == 0) continue;
        const int bw = jacobi_bw(r, lds_elems, sizeof(R) == 8 ? 2 : 1);
        const int nb = (r + bw - 1) / bw;
        const int ne = (nb + 1) & ~1;
        if ((int)rounds.size() < ne - 1) rounds.resize(ne - 1);
        for (int t = 0; t < ne - 1; ++t)
            for (int pr = 0; pr < ne / 2; ++pr) {
                const int bi = rr_slot_host(pr, t, ne), bj = rr_slot_host(ne - 1 - pr, t, ne);
                if (bi < nb && bj < nb) rounds[t].push_back({s, bi, bj, 0});
            }
    }
    std::vector<JacTask> all;
    std::vector<size_t> t0;
    for (const auto &rt : rounds) {
        t0.push_back(all.size());
        all.insert(all.end(), rt.begin(), rt.end());
    }
    std::vector<int32_t> active(nbig), rot(nbig);
    for (int s = 0; s < nbig; ++s) active[s] = blk[order[q0 + s]].r > 0;
    if (!all.empty()) {
        d_tasks.alloc(all.size() * sizeof(JacTask));
        HM_HIP_CHECK(hipMemcpyAsync(d_tasks.p, all.data(), all.size() * sizeof(JacTask),
                                    hipMemcpyHostToDevice, st));
        for (int sweep = 0; sweep < 30; ++sweep) {
            HM_HIP_CHECK(hipMemcpyAsync(d_active.p, active.data(), nbig * sizeof(int32_t),
                                        hipMemcpyHostToDevice, st));
            HM_HIP_CHECK(hipMemsetAsync(d_rot.p, 0, nbig * sizeof(int32_t), st));
            for (size_t t = 0; t < rounds.size(); ++t)
                if (!rounds[t].empty())
                    hipLaunchKernelGGL(jacobi_round_kernel<sizeof(R) == 8>,
                                       dim3((unsigned)rounds[t].size()),
                                       dim3(1024), bytes, st, d_blk, d_order + q0,
                                       d_tasks.as<JacTask>() + t0[t], W, d_tiny.as<double>(),
                                       d_active.as<int32_t>(), d_rot.as<int32_t>(), lds_elems);
            HM_HIP_CHECK(hipGetLastError());
            HM_HIP_CHECK(hipMemcpyAsync(rot.data(), d_rot.p, nbig * sizeof(int32_t),
                                        hipMemcpyDeviceToHost, st));
            HM_HIP_CHECK(hipStreamSynchronize(st));
            bool any = false;
            for (int s = 0; s < nbig; ++s) {
                active[s] = active[s] && rot[s];
                any = any || active[s];
            }
            if (!any) break;
        }
    }
    hipLaunchKernelGGL((factor_kernel<R, 1024, 2>), dim3((unsigned)nbig), dim3(1024), bytes, st,
                       d_blk, d_order + q0, W, d_newrank, eps, lds_elems, nullptr);
    HM_HIP_CHECK(hipGetLastError());
    // the host vectors above outlive their copies
    HM_HIP_CHECK(hipStreamSynchronize(st));
}

template <typename R>
void run_recompress(const std::vector<RcBlk> &blk, RcBlk *d_blk, const cplx<R> *acaslab,
                    double *work, int32_t *d_newrank, double eps, int32_t rmax, hipStream_t st,
                    bool unbatched, bool wide_small) {
    if (blk.empty()) return;
    std::vector<GramItem> items;
    std::vector<int64_t> item0(blk.size() + 1, 0);   // items of block i: item0[i] .. item0[i+1]
    for (int32_t i = 0; i < (int32_t)blk.size(); ++i) {
        const int T = (int)ceil_div(blk[i].r, kGT);
        for (int w = 0; w < 2; ++w)
            for (int a = 0; a < T; ++a)
                for (int c = a; c < T; ++c) items.push_back({i, w, a, c});
        item0[i + 1] = (int64_t)items.size();
    }
    (void)rmax;
    DeviceBuf d_items;
    if (!items.empty()) {
        d_items.alloc(items.size() * sizeof(GramItem));
        HM_HIP_CHECK(hipMemcpyAsync(d_items.p, items.data(), items.size() * sizeof(GramItem),
                                    hipMemcpyHostToDevice, st));
        if (unbatched) {
            for (size_t i = 0; i < blk.size(); ++i)
                if (item0[i + 1] > item0[i])
                    hipLaunchKernelGGL(gram_mfma_kernel<R>, dim3((unsigned)(item0[i + 1] - item0[i])),
                                       dim3(256), 0, st, d_blk, d_items.as<GramItem>() + item0[i],
                                       acaslab, reinterpret_cast<cplx<double> *>(work));
        } else {
            hipLaunchKernelGGL(gram_mfma_kernel<R>, dim3((unsigned)items.size()), dim3(256), 0, st,
                               d_blk, d_items.as<GramItem>(), acaslab,
                               reinterpret_cast<cplx<double> *>(work));
        }
        HM_HIP_CHECK(hipGetLastError());
    }
    // LDS for the Jacobi sweeps: per rank class, what M and J of the largest
    // block of the class need (whole-matrix mode), capped at what the device
    // grants one workgroup (block mode above that), so that small blocks keep
    // several workgroups per CU.
    int max_lds = 0;
    {
        int dev = 0, v = 65536;
        HM_HIP_CHECK(hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
        max_lds = std::min(v, 160 * 1024) - 1024;
        if (max_lds > 65536) {
            const void *kerns[] = {(const void *)factor_kernel<R, 256, 0>,
                                   (const void *)factor_kernel<R, 1024, 0>,
                                   (const void *)factor_kernel<R, 1024, 1>,
                                   (const void *)factor_kernel<R, 1024, 2>,
                                   (const void *)jacobi_round_kernel<false>,
                                   (const void *)jacobi_round_kernel<true>};
            for (const void *k : kerns)
                HM_HIP_CHECK(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 max_lds));
        }
    }
    std::vector<int32_t> order(blk.size());
    for (size_t i = 0; i < blk.size(); ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return blk[a].r > blk[b].r; });
    DeviceBuf d_order;
    d_order.alloc(order.size() * sizeof(int32_t));
    HM_HIP_CHECK(hipMemcpyAsync(d_order.p, order.data(), order.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, st));
    const int classes[] = {16, 24, 32, 48, 64, 100, 1 << 30};
    // The classes of ranks above 64 run one workgroup per CU and leave CUs
    // idle; the smaller classes go to a second stream and fill them.  When
    // some cores are too large for LDS, their split sweeps hold the build
    // stream, and every other class goes to the second stream.
    hipStream_t side = st;
    ScopedEvent ev_ready, ev_done;
    if (!unbatched) {
        side = side_stream(0);
        HM_HIP_CHECK(hipEventRecord(ev_ready.e, st));   // gram products and d_order are queued
        HM_HIP_CHECK(hipStreamWaitEvent(side, ev_ready.e, 0));
    }
    struct {
        size_t q0 = 0, q1 = 0, bytes = 0;
        int64_t lds_elems = 0;
    } split;
    size_t q0 = 0;
    while (q0 < order.size()) {
        const int rmax = blk[order[q0]].r;
        int cls = 0;
        while (classes[cls] < rmax) ++cls;
        const int lo = cls > 0 ? classes[cls - 1] : -1;
        size_t q1 = q0;
        while (q1 < order.size() && blk[order[q1]].r > lo) ++q1;
        // complex128 sweeps carry J beside M (twice the LDS for in-LDS sweeps)
        const int64_t need = (int64_t)rmax * rmax * (int64_t)sizeof(cplx<double>);
        const int64_t bytes = std::min<int64_t>(sizeof(R) == 8 ? 2 * need : need, max_lds);
        const int64_t lds_elems = bytes / (int64_t)sizeof(cplx<double>);
        // ranks above 64 leave room for one workgroup per CU (LDS): give it
        // 1024 threads (more lanes per Jacobi pair and per Cholesky column)
        // (wide_small: every class, for callers with few blocks per call)
        const bool wide = rmax > 64 || wide_small;
        auto kern = wide ? factor_kernel<R, 1024, 0> : factor_kernel<R, 256, 0>;
        const unsigned nt = wide ? 1024u : 256u;
        if (unbatched) {
            for (size_t q = q0; q < q1; ++q)
                hipLaunchKernelGGL(kern, dim3(1), dim3(nt), (size_t)bytes, st, d_blk,
                                   d_order.as<int32_t>() + q,
                                   reinterpret_cast<cplx<double> *>(work), d_newrank, eps,
                                   lds_elems, nullptr);
        } else if ((int64_t)rmax * rmax <= lds_elems) {
            hipLaunchKernelGGL(kern, dim3((unsigned)(q1 - q0)), dim3(nt), (size_t)bytes,
                               split.q1 > split.q0 || rmax <= 64 ? side : st, d_blk,
                               d_order.as<int32_t>() + q0,
                               reinterpret_cast<cplx<double> *>(work), d_newrank, eps, lds_elems,
                               nullptr);
        } else {
            // after the other classes are queued: its host loop waits on the GPU
            split = {q0, q1, (size_t)bytes, lds_elems};
        }
        HM_HIP_CHECK(hipGetLastError());
        q0 = q1;
    }
    if (split.q1 > split.q0)
        split_jacobi<R>(blk, order, split.q0, split.q1, d_blk, d_order.as<int32_t>(), work,
                        d_newrank, eps, split.bytes, split.lds_elems, st);
    if (!unbatched) {
        HM_HIP_CHECK(hipEventRecord(ev_done.e, side));
        HM_HIP_CHECK(hipStreamWaitEvent(st, ev_done.e, 0));
        HM_HIP_CHECK(hipStreamSynchronize(st));
    }
    HM_HIP_CHECK(hipGetLastError());
    // items (pageable) and d_items must outlive the copy and the kernels.
    HM_HIP_CHECK(hipStreamSynchronize(st));
}

template <typename R>
void run_recompress_apply(const std::vector<RcBlk> &blk, RcBlk *d_blk, const cplx<R> *acaslab,
                          const double *work, const int64_t *d_outu, const int64_t *d_outv,
                          const int32_t *d_newrank, cplx<R> *out, const std::vector<int32_t> &keep,
                          const int32_t *d_rowpad, hipStream_t st, bool unbatched) {
    if (blk.empty()) return;
    std::vector<ApplyTask> tasks;
    std::vector<int64_t> task0(blk.size() + 1, 0);
    for (int32_t i = 0; i < (int32_t)blk.size(); ++i) {
        if (keep[i] != 0)
            for (int w = 0; w < 2; ++w) {
                const int32_t rows = 3 * (w == 0 ? blk[i].m : blk[i].n);
                for (int32_t r0 = 0; r0 < rows; r0 += 64)
                    for (int32_t c0 = 0; c0 < keep[i]; c0 += 64) tasks.push_back({i, w, r0, c0});
            }
        task0[i + 1] = (int64_t)tasks.size();
    }
    if (tasks.empty()) return;
    DeviceBuf d_tasks;
    d_tasks.alloc(tasks.size() * sizeof(ApplyTask));
    HM_HIP_CHECK(hipMemcpyAsync(d_tasks.p, tasks.data(), tasks.size() * sizeof(ApplyTask),
                                hipMemcpyHostToDevice, st));
    if (unbatched) {
        for (size_t i = 0; i < blk.size(); ++i)
            if (task0[i + 1] > task0[i])
                hipLaunchKernelGGL(apply_kernel<R>, dim3((unsigned)(task0[i + 1] - task0[i])),
                                   dim3(256), 0, st, d_blk, d_tasks.as<ApplyTask>() + task0[i],
                                   acaslab, reinterpret_cast<const cplx<double> *>(work),
                                   d_newrank, d_outu, d_outv, out, d_rowpad);
    } else {
        hipLaunchKernelGGL(apply_kernel<R>, dim3((unsigned)tasks.size()), dim3(256), 0, st, d_blk,
                           d_tasks.as<ApplyTask>(), acaslab,
                           reinterpret_cast<const cplx<double> *>(work), d_newrank, d_outu,
                           d_outv, out, d_rowpad);
    }
    HM_HIP_CHECK(hipGetLastError());
    // tasks (pageable) and d_tasks must outlive the copy and the kernel
    HM_HIP_CHECK(hipStreamSynchronize(st));
}

template void run_recompress<float>(const std::vector<RcBlk> &, RcBlk *, const cplx<float> *,
                                    double *, int32_t *, double, int32_t, hipStream_t, bool, bool);
template void run_recompress<double>(const std::vector<RcBlk> &, RcBlk *, const cplx<double> *,
                                     double *, int32_t *, double, int32_t, hipStream_t, bool, bool);
template void run_recompress_apply<float>(const std::vector<RcBlk> &, RcBlk *,
                                          const cplx<float> *, const double *, const int64_t *,
                                          const int64_t *, const int32_t *, cplx<float> *,
                                          const std::vector<int32_t> &, const int32_t *,
                                          hipStream_t, bool);
template void run_recompress_apply<double>(const std::vector<RcBlk> &, RcBlk *,
                                           const cplx<double> *, const double *, const int64_t *,
                                           const int64_t *, const int32_t *, cplx<double> *,
                                           const std::vector<int32_t> &, const int32_t *,
                                           hipStream_t, bool);

}  // namespace hm
