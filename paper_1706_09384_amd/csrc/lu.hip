// H-LU factorisation and solve (Section 3.2) and the quantities of the
// certification estimator (Section 3.3, eq. est_direct), complex128.
//
// The factorisation runs the recursive 2 x 2 block LU over the block
// cluster tree on the host, as a sequence of device operations on one
// stream: every block of the factors is dense (F, column-major), low-rank
// (R, U W with W = V^*, both column-major) or subdivided (H).  The device
// work is
//   * dense diagonal leaves: elimination without pivoting in one workgroup
//     (lu_getrf_kernel), then the inverses of both triangular factors, one
//     column per thread over several workgroups (lu_trinv_kernel);
//   * every product (block substitutions against a diagonal leaf are
//     products with its inverse factors, low-rank products, dense updates):
//     a strided complex FP64 matrix-core GEMM (lu_gemm_kernel);
//   * sums into a low-rank block are kept exactly as extra factor columns
//     and recompressed at eps_LU, in batches over all the blocks that one
//     block substitution is about to read, with the assembly's
//     QR + truncated SVD kernels.
// Device memory comes from two arenas: one for the factors and the pending
// low-rank pieces (freed with the object), one stack for temporaries
// (released in stream order).
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <memory>
#include <map>
#include <vector>

#include "green.hpp"
#include "internal.hpp"
#include "lu_core.hpp"
#include "mfma_gemm.hpp"
#include "rng.hpp"

namespace hm {

using Z = cplx<double>;
using lu::DMat;
using lu::LuNode;
using lu::need;

namespace {

__host__ __device__ inline Z zdiv(Z a, Z b) {
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// ------------------------------------------------------------------ kernels

// C = alpha A B (+ C when beta), element (i, j) of X at X[i rs + j cs]:
// 64 x 64 output tiles per workgroup, the four waves on its 32 x 32
// quadrants (2 x 2 tiles of v_mfma_f64_16x16x4f64 each), 16-deep slabs of A
// and B staged in LDS along whichever index is contiguous in memory.
struct GemmArgs {
    const Z *A;
    int64_t ars, acs;
    const Z *B;
    int64_t brs, bcs;
    Z *C;
    int64_t crs, ccs;
    int32_t m, n, k;
    Z alpha;
    int32_t beta;
    int32_t conja, conjb;   // use conj(A) / conj(B) entries
    int32_t kchunk;         // split-K: slice z of the grid sums k in [z kchunk, (z + 1) kchunk)
    int64_t zstride;        // and writes its partial product at C + z zstride
};

__global__ void __launch_bounds__(256) lu_gemm_kernel(GemmArgs g) {
    constexpr int kT = 64, kS = 16;
    __shared__ Z sa[kS][kT + 1], sb[kS][kT + 1];
    const int i0 = blockIdx.x * kT, j0 = blockIdx.y * kT;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wa = wave & 1, wb = wave >> 1, gq = lane >> 4, l16 = lane & 15;
    // three real products per complex one: P1 = Re a Re b, P2 = Im a Im b,
    // P3 = (Re a + Im a)(Re b + Im b); Re = P1 - P2, Im = P3 - P1 - P2
    mf64x4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) p1[i][j] = p2[i][j] = p3[i][j] = mf64x4{0, 0, 0, 0};
    const bool a_rows = g.ars == 1, b_rows = g.brs == 1;
    const int kb = blockIdx.z * g.kchunk, ke = min(g.k, kb + g.kchunk);
    for (int k0 = kb; k0 < ke; k0 += kS) {
        for (int e = tid; e < kS * kT; e += 256) {
            int i, kk;
            if (a_rows) { i = e % kT; kk = e / kT; } else { kk = e % kS; i = e / kS; }
            Z av = (i0 + i < g.m && k0 + kk < ke)
                       ? g.A[(int64_t)(i0 + i) * g.ars + (int64_t)(k0 + kk) * g.acs]
                       : Z{0, 0};
            if (g.conja) av.im = -av.im;
            sa[kk][i] = av;
            int j, k2;
            if (b_rows) { k2 = e % kS; j = e / kS; } else { j = e % kT; k2 = e / kT; }
            Z bv = (k0 + k2 < ke && j0 + j < g.n)
                       ? g.B[(int64_t)(k0 + k2) * g.brs + (int64_t)(j0 + j) * g.bcs]
                       : Z{0, 0};
            if (g.conjb) bv.im = -bv.im;
            sb[k2][j] = bv;
        }
        __syncthreads();
#pragma unroll
        for (int s4 = 0; s4 < kS; s4 += 4) {
            Z A[2], B[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                A[t] = sa[s4 + gq][32 * wa + 16 * t + l16];
                B[t] = sb[s4 + gq][32 * wb + 16 * t + l16];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    p1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[i].re, B[j].re, p1[i][j], 0, 0, 0);
                    p2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[i].im, B[j].im, p2[i][j], 0, 0, 0);
                    p3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[i].re + A[i].im,
                                                                    B[j].re + B[j].im, p3[i][j], 0, 0, 0);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = i0 + 32 * wa + 16 * i + 4 * e + gq;
                const int col = j0 + 32 * wb + 16 * j + l16;
                if (row < g.m && col < g.n) {
                    const Z v = {p1[i][j][e] - p2[i][j][e], p3[i][j][e] - p1[i][j][e] - p2[i][j][e]};
                    Z *c = g.C + blockIdx.z * g.zstride + (int64_t)row * g.crs + (int64_t)col * g.ccs;
                    const Z r = g.alpha * v;
                    *c = g.beta ? *c + r : r;
                }
            }
}

// dst(i, j) = [dst(i, j) +] alpha op(src(i, j)), op = conj when cj.
__global__ void lu_copy_kernel(Z *dst, int64_t drs, int64_t dcs, const Z *src, int64_t srs,
                               int64_t scs, int32_t m, int32_t n, Z alpha, int32_t cj,
                               int32_t acc) {
    const int64_t tot = (int64_t)m * n;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q % m, j = q / m;
        Z v = src[i * srs + j * scs];
        if (cj) v = conj(v);
        v = alpha * v;
        Z *d = dst + i * drs + j * dcs;
        *d = acc ? *d + v : v;
    }
}

// C(i, j) = [C(i, j) +] sum_z P_z(i, j), the split-K partials (m x n,
// column-major, z = 0 .. nz - 1 in order).
__global__ void lu_ksum_kernel(Z *dst, int64_t drs, int64_t dcs, const Z *__restrict__ P, int32_t m,
                               int32_t n, int32_t nz, int32_t acc) {
    const int64_t tot = (int64_t)m * n;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot;
         q += (int64_t)gridDim.x * blockDim.x) {
        Z v = {0, 0};
        for (int z = 0; z < nz; ++z) v = v + P[z * tot + q];
        Z *d = dst + (q % m) * drs + (q / m) * dcs;
        *d = acc ? *d + v : v;
    }
}

// dst(i, j) = (i == j ? diag : 0).
__global__ void lu_fill_kernel(Z *dst, int64_t drs, int64_t dcs, int32_t m, int32_t n, Z diag) {
    const int64_t tot = (int64_t)m * n;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q % m, j = q / m;
        dst[i * drs + j * dcs] = i == j ? diag : Z{0, 0};
    }
}

// om[e] = gauss_at(seed, e), e < count.
__global__ void lu_gauss_kernel(Z *__restrict__ om, int64_t count, uint64_t seed) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        om[e] = gauss_at(seed, (uint64_t)e);
}

// Per item: Re sum_e a[e] conj(b[e]) over `count` entries, one workgroup each.
struct DotItem {
    const Z *a, *b;
    int64_t count;
};

__device__ inline double wave_sum_lu(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(256) lu_dot_kernel(const DotItem *__restrict__ items,
                                                     double *__restrict__ out) {
    const DotItem it = items[blockIdx.x];
    double s = 0;
    for (int64_t e = threadIdx.x; e < it.count; e += 256) {
        const Z x = it.a[e], y = it.b[e];
        s += x.re * y.re + x.im * y.im;
    }
    __shared__ double red[4];
    s = wave_sum_lu(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Dense tile of the H-matrix (padded leaf-segment rows, storage type S) to a
// plain column-major complex128 array of 3m rows.
template <typename S>
__global__ void lu_import_dense_kernel(const cplx<S> *__restrict__ src, int64_t ld,
                                       const int32_t *__restrict__ rowpad, int32_t rb, int32_t m,
                                       int32_t ncols, Z *__restrict__ dst) {
    const int64_t rows = 3 * (int64_t)m, tot = rows * ncols;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = q % rows, c = q / rows;
        dst[q] = cvt<double>(src[c * ld + padded_row(rowpad, rb, (int32_t)(row / 3), (int)(row % 3))]);
    }
}

// Low-rank block U V^* of the H-matrix (U padded column-major, V row-major)
// to U (3m x r) and W = V^* (r x 3n), column-major complex128.
template <typename S>
__global__ void lu_import_lr_kernel(const cplx<S> *__restrict__ U, int64_t ldu,
                                    const cplx<S> *__restrict__ V, int64_t ldv,
                                    const int32_t *__restrict__ rowpad, int32_t rb, int32_t m,
                                    int32_t n, int32_t r, Z *__restrict__ Uo, Z *__restrict__ Wo) {
    const int64_t mr = 3 * (int64_t)m, nr = 3 * (int64_t)n;
    const int64_t tot = (mr + nr) * r;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot;
         q += (int64_t)gridDim.x * blockDim.x) {
        if (q < mr * r) {
            const int64_t row = q % mr, c = q / mr;
            Uo[q] = cvt<double>(U[c * ldu + padded_row(rowpad, rb, (int32_t)(row / 3), (int)(row % 3))]);
        } else {
            const int64_t e = q - mr * r;
            const int64_t c = e % r, j = e / r;
            Wo[e] = conj(cvt<double>(V[j * ldv + c]));
        }
    }
}

// In place: A (n x n, column-major) = L \ U by elimination without pivoting
// (unit lower L).  One workgroup.
__global__ void __launch_bounds__(1024) lu_getrf_kernel(Z *__restrict__ A, int32_t n,
                                                        int32_t *__restrict__ zero_pivot) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int k = 0; k < n; ++k) {
        const Z piv = A[k + (int64_t)k * n];
        if (piv.re == 0.0 && piv.im == 0.0) {
            if (tid == 0) atomicAdd(zero_pivot, 1);
            return;   // uniform: every thread read the same pivot
        }
        const Z inv = zdiv(Z{1, 0}, piv);
        for (int i = k + 1 + tid; i < n; i += nt) A[i + (int64_t)k * n] = A[i + (int64_t)k * n] * inv;
        __syncthreads();
        const int rem = n - k - 1;
        for (int q = tid; q < rem * rem; q += nt) {
            const int i = k + 1 + q % rem, j = k + 1 + q / rem;
            const Z l = A[i + (int64_t)k * n], u = A[k + (int64_t)j * n];
            Z &a = A[i + (int64_t)j * n];
            a = a - l * u;
        }
        __syncthreads();
    }
}

// Linv = L^-1 (blockIdx.y = 0) and Uinv = U^-1 (blockIdx.y = 1) of the
// factored A by substitution, one column per thread, the columns spread over
// workgroups of 64.  (After a zero pivot the host discards the result.)
__global__ void __launch_bounds__(64) lu_trinv_kernel(const Z *__restrict__ A, Z *__restrict__ Linv,
                                                      Z *__restrict__ Uinv, int32_t n) {
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (j >= n) return;
    if (blockIdx.y == 0) {
        Z *x = Linv + (int64_t)j * n;
        for (int i = 0; i < j; ++i) x[i] = Z{0, 0};
        x[j] = Z{1, 0};
        for (int i = j + 1; i < n; ++i) {
            Z s = {0, 0};
            for (int k = j; k < i; ++k) fma_(s, A[i + (int64_t)k * n], x[k]);
            x[i] = Z{-s.re, -s.im};
        }
    } else {
        Z *y = Uinv + (int64_t)j * n;
        for (int i = j + 1; i < n; ++i) y[i] = Z{0, 0};
        for (int i = j; i >= 0; --i) {
            Z s = i == j ? Z{1, 0} : Z{0, 0};
            for (int k = i + 1; k <= j; ++k) s = s - A[i + (int64_t)k * n] * y[k];
            y[i] = zdiv(s, A[i + (int64_t)i * n]);
        }
    }
}

// b (original point order, row-major (3N, nrhs)) -> X (cluster order,
// column-major 3N x nrhs), and back.
__global__ void lu_gather_kernel(const Z *__restrict__ b, const int32_t *__restrict__ perm,
                                 int64_t dofs, int32_t nrhs, Z *__restrict__ X) {
    const int64_t tot = dofs * nrhs;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q % dofs, c = q / dofs;
        X[q] = b[(3 * (int64_t)perm[i / 3] + i % 3) * nrhs + c];
    }
}

__global__ void lu_scatter_kernel(const Z *__restrict__ X, const int32_t *__restrict__ perm,
                                  int64_t dofs, int32_t nrhs, Z *__restrict__ x) {
    const int64_t tot = dofs * nrhs;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < tot;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q % dofs, c = q / dofs;
        x[(3 * (int64_t)perm[i / 3] + i % 3) * nrhs + c] = X[q];
    }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

unsigned grid_for(int64_t tot) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(tot, 256), 65536)); }

// ------------------------------------------------------------------ memory

// Bump allocator over device chunks; mark / release give stack discipline
// for temporaries (reuse is safe in stream order: a later kernel on the same
// stream runs after every kernel that used the memory before).
struct Arena {
    std::vector<std::unique_ptr<DeviceBuf>> chunks;
    std::vector<size_t> caps;
    int cur = -1;
    size_t used = 0;
    size_t chunk_bytes;
    size_t total = 0;
    explicit Arena(size_t cb) : chunk_bytes(cb) {}
    struct Mark {
        int cur;
        size_t used;
    };
    Mark mark() const { return {cur, used}; }
    void release(Mark m) {
        cur = m.cur;
        used = m.used;
    }
    Z *alloc(int64_t elems) {
        const size_t b = std::max<size_t>(256, ((size_t)std::max<int64_t>(elems, 1) * sizeof(Z) + 255) & ~size_t(255));
        if (cur >= 0 && used + b <= caps[cur]) {
            Z *p = reinterpret_cast<Z *>(static_cast<char *>(chunks[cur]->p) + used);
            used += b;
            return p;
        }
        for (int c = cur + 1; c < (int)chunks.size(); ++c)
            if (caps[c] >= b) {
                cur = c;
                used = b;
                return chunks[c]->as<Z>();
            }
        auto buf = std::make_unique<DeviceBuf>();
        const size_t cb = std::max(chunk_bytes, b);
        buf->alloc(cb);
        total += cb;
        chunks.push_back(std::move(buf));
        caps.push_back(cb);
        cur = (int)chunks.size() - 1;
        used = b;
        return chunks.back()->as<Z>();
    }
    Z *base() const { return chunks.empty() ? nullptr : chunks[0]->as<Z>(); }
};

}  // namespace
}  // namespace hm

struct hm_lu {
    double eps = 0;
    int64_t dofs = 0;
    std::vector<hm::lu::LuNode> nodes;
    hm::Arena keep{size_t(1) << 28};
    // freed keep memory by size class (bytes), handed out again by keep_alloc
    std::map<size_t, std::vector<hm::cplx<double> *>> keep_pool;
    hm::Arena tmp{size_t(1) << 28};   // stack of the caller's stream (factor, solve, export)
    hm::DeviceBuf d_perm, d_zero_rowpad, d_flag;
    hm_lu_stats stats{};
    hipStream_t st = nullptr;
    uint64_t rng_calls = 0;   // counter of the range finder's Gaussian draws
};

namespace hm {
namespace {

// Keep memory that may be freed and reused comes in size classes (the size
// rounded up to 8 steps per power of two, at least 256 bytes), so that memory
// freed by one block's recompression serves later requests of the same class.
size_t keep_class(int64_t n) {
    const size_t b = std::max<size_t>(256, (size_t)std::max<int64_t>(n, 1) * sizeof(Z));
    const int e = 63 - __builtin_clzll((unsigned long long)b);
    const size_t step = std::max<size_t>(256, size_t(1) << std::max(e - 3, 0));
    return (b + step - 1) / step * step;
}
// The smallest freed block of class c to 2c serves a request of class c (a
// larger block goes back under the class of the request it served: it is
// then only handed out for requests it covers).
Z *keep_class_alloc(hm_lu &F, int64_t n) {
    const size_t c = keep_class(n);
    for (auto it = F.keep_pool.lower_bound(c); it != F.keep_pool.end() && it->first <= 2 * c; ++it)
        if (!it->second.empty()) {
            Z *p = it->second.back();
            it->second.pop_back();
            return p;
        }
    return F.keep.alloc((int64_t)(c / sizeof(Z)));
}

// Streams the factorisation spreads independent branches over: the caller's
// stream and up to kLuStreams - 1 more.
constexpr int kLuStreams = 4;

// The H-LU's arithmetic on the device: kernels of this file, and the
// assembly's QR + truncated SVD for the eps_LU recompressions.
//
// Independent branches of the recursion (fork / branch / join) run on
// different streams: branch b of a fork taken on stream p goes to stream
// (p + b) mod n, which first waits for an event recorded on p at the fork; at
// the join p waits for an event recorded on every stream a branch used.  Each
// stream has a stack arena of its own, and a branch allocates only from its
// stream's arena, so stack memory is reused only in the order of the stream
// that used it, or after a join that ordered every user before the reuse.
// Every kernel's operands are the same whatever the schedule, so the factors
// do not depend on the number of streams.
struct GpuBackend {
    hm_lu &F;
    hipStream_t st;   // current stream
    int cur = 0, nstreams = 1;
    hipStream_t strm[kLuStreams] = {};
    Arena *arena[kLuStreams] = {};
    std::vector<hipEvent_t> *events = nullptr;   // owned by the caller, destroyed after a sync

    GpuBackend(hm_lu &f, hipStream_t s) : F(f), st(s) {
        strm[0] = s;
        arena[0] = &f.tmp;
    }
    Arena &tmp() { return *arena[cur]; }
    struct Mark {
        int a;
        Arena::Mark m;
    };

    Z *keep_alloc(int64_t n) { return keep_class_alloc(F, n); }
    // keep_free is called once no kernel will touch the memory again (after a
    // truncate, which drains its stream, and every stream that wrote the
    // memory was joined into that one before), so reuse needs no ordering
    void keep_free(Z *p, int64_t n) {
        if (p) F.keep_pool[keep_class(n)].push_back(p);
    }
    Z *tmp_alloc(int64_t n) { return tmp().alloc(n); }
    Mark tmp_mark() { return {cur, tmp().mark()}; }
    void tmp_release(Mark m) { arena[m.a]->release(m.m); }
    hm_lu_stats &stats() { return F.stats; }

    struct Fork {
        int parent;
        hipEvent_t ev;
        unsigned used;
    };
    hipEvent_t new_event() {
        hipEvent_t e = nullptr;
        HM_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        events->push_back(e);
        return e;
    }
    Fork fork() {
        Fork f{cur, nullptr, 0u};
        if (nstreams > 1) {
            f.ev = new_event();
            HM_HIP_CHECK(hipEventRecord(f.ev, strm[cur]));
        }
        return f;
    }
    void branch(Fork &f, int b) {
        const int s = (f.parent + b) % nstreams;
        if (s != f.parent && !((f.used >> s) & 1u)) {
            HM_HIP_CHECK(hipStreamWaitEvent(strm[s], f.ev, 0));
            f.used |= 1u << s;
        }
        cur = s;
        st = strm[s];
    }
    void join(Fork &f) {
        for (int s = 0; s < nstreams; ++s)
            if ((f.used >> s) & 1u) {
                hipEvent_t e = new_event();
                HM_HIP_CHECK(hipEventRecord(e, strm[s]));
                HM_HIP_CHECK(hipStreamWaitEvent(strm[f.parent], e, 0));
            }
        cur = f.parent;
        st = strm[cur];
    }

    void gemm(DMat C, DMat A, DMat B, Z alpha, bool beta) { gemm_c(C, A, false, B, false, alpha, beta); }
    // C = alpha op(A) op(B) (+ C), op = conj when the flag is set
    void gemm_c(DMat C, DMat A, bool ca, DMat B, bool cb, Z alpha, bool beta) {
        need(A.m == C.m && B.n == C.n && A.n == B.m, "H-LU: product shapes");
        if (C.m == 0 || C.n == 0) return;
        const int64_t tiles = ceil_div(C.m, 64) * ceil_div(C.n, 64);
        // few output tiles over a long inner dimension: split the inner
        // dimension over the grid's z slices into partial products summed in
        // slice order afterwards (deterministic)
        int32_t nz = 1;
        if (tiles < 64 && A.n >= 1024)
            nz = (int32_t)std::min<int64_t>({A.n / 256, std::max<int64_t>(1, 256 / tiles), 64});
        if (nz <= 1) {
            GemmArgs g{A.p, A.rs, A.cs, B.p, B.rs, B.cs, C.p, C.rs, C.cs, C.m, C.n, A.n, alpha,
                       beta ? 1 : 0, ca ? 1 : 0, cb ? 1 : 0, A.n, 0};
            hipLaunchKernelGGL(lu_gemm_kernel, dim3((unsigned)ceil_div(C.m, 64), (unsigned)ceil_div(C.n, 64)),
                               dim3(256), 0, st, g);
            HM_HIP_CHECK(hipGetLastError());
            return;
        }
        const int32_t kchunk = (int32_t)(ceil_div(ceil_div(A.n, nz), 16) * 16);
        nz = (int32_t)ceil_div(A.n, kchunk);
        Arena &ar = tmp();
        const auto mk = ar.mark();
        const int64_t mn = (int64_t)C.m * C.n;
        Z *P = ar.alloc(mn * nz);
        GemmArgs g{A.p, A.rs, A.cs, B.p, B.rs, B.cs, P, 1, C.m, C.m, C.n, A.n, alpha,
                   0, ca ? 1 : 0, cb ? 1 : 0, kchunk, mn};
        hipLaunchKernelGGL(lu_gemm_kernel,
                           dim3((unsigned)ceil_div(C.m, 64), (unsigned)ceil_div(C.n, 64), (unsigned)nz),
                           dim3(256), 0, st, g);
        hipLaunchKernelGGL(lu_ksum_kernel, dim3(grid_for(mn)), dim3(256), 0, st, C.p, C.rs, C.cs, P,
                           C.m, C.n, nz, beta ? 1 : 0);
        HM_HIP_CHECK(hipGetLastError());
        ar.release(mk);
    }
    // Re sum a conj(b) per item (synchronous)
    std::vector<double> dots(const std::vector<DotItem> &items) {
        std::vector<double> out(items.size());
        if (items.empty()) return out;
        DeviceBuf d_items, d_out;
        d_items.alloc(items.size() * sizeof(DotItem));
        d_out.alloc(items.size() * sizeof(double));
        HM_HIP_CHECK(hipMemcpyAsync(d_items.p, items.data(), items.size() * sizeof(DotItem),
                                    hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(lu_dot_kernel, dim3((unsigned)items.size()), dim3(256), 0, st,
                           d_items.as<DotItem>(), d_out.as<double>());
        HM_HIP_CHECK(hipGetLastError());
        HM_HIP_CHECK(hipMemcpyAsync(out.data(), d_out.p, out.size() * sizeof(double),
                                    hipMemcpyDeviceToHost, st));
        HM_HIP_CHECK(hipStreamSynchronize(st));
        return out;
    }
    // Randomized range finder (Liberty, Woolfe, Martinsson, Rokhlin and Tygert
    // 2007) in front of the recompression of wide stacks: for B = U V^* with
    // K > kRandMinK columns, Y = B Omega (s complex Gaussian columns), Q =
    // orth(Y), Z = B^* Q, accepted when |B|_F^2 - |Z|_F^2 = |B - Q Q^* B|_F^2
    // <= (eps / 2)^2 |B|_F^2 (s doubles otherwise, up to kRsMaxK and below K);
    // an accepted item continues as (Q, Z) with s columns.  The recompression
    // then truncates at eps as before; the Jacobi core shrinks from K to s.
    static constexpr int32_t kRandMinK = 64;
    void range_finder(std::vector<lu::RcItem> &items, double eps) {
        std::vector<size_t> act;
        for (size_t i = 0; i < items.size(); ++i)
            if (items[i].K > kRandMinK) act.push_back(i);
        if (act.empty()) return;
        const auto cm_ = [](Z *p, int32_t m, int32_t n) { return lu::cm(p, m, n, std::max(m, 1)); };
        const auto adj = [](DMat X) { return DMat{X.p, X.cs, X.rs, X.n, X.m}; };   // X^T (use with conj)
        // |B|_F^2 = sum_ij (U^* U)_ij conj((V^* V)_ij)
        std::vector<DotItem> di;
        for (size_t a : act) {
            const lu::RcItem &it = items[a];
            DMat U = cm_(it.U, it.m, it.K), V = cm_(it.V, it.n, it.K);
            DMat GU = cm_(tmp().alloc((int64_t)it.K * it.K), it.K, it.K);
            DMat GV = cm_(tmp().alloc((int64_t)it.K * it.K), it.K, it.K);
            gemm_c(GU, adj(U), true, U, false, Z{1, 0}, false);
            gemm_c(GV, adj(V), true, V, false, Z{1, 0}, false);
            di.push_back({GU.p, GV.p, (int64_t)it.K * it.K});
        }
        const std::vector<double> nb = dots(di);
        std::vector<int32_t> s(act.size());
        for (size_t a = 0; a < act.size(); ++a) s[a] = std::min(items[act[a]].K, kRandMinK);
        std::vector<size_t> live(act.size());
        for (size_t a = 0; a < act.size(); ++a) live[a] = a;
        Z *base = F.keep.base();
        while (!live.empty()) {
            std::vector<DMat> Q(live.size()), Zm(live.size());
            std::vector<RsBlk> ob(live.size());
            for (size_t l = 0; l < live.size(); ++l) {
                const lu::RcItem &it = items[act[live[l]]];
                const int32_t k = s[live[l]];
                DMat U = cm_(it.U, it.m, it.K), V = cm_(it.V, it.n, it.K);
                DMat Om = cm_(tmp().alloc((int64_t)it.n * k), it.n, k);
                hipLaunchKernelGGL(lu_gauss_kernel, dim3(grid_for((int64_t)it.n * k)), dim3(256), 0, st, Om.p,
                                   (int64_t)it.n * k, 0x9E3779B97F4A7C15ull * (++F.rng_calls));
                HM_HIP_CHECK(hipGetLastError());
                DMat T = cm_(tmp().alloc((int64_t)it.K * k), it.K, k);
                gemm_c(T, adj(V), true, Om, false, Z{1, 0}, false);       // V^* Omega
                Q[l] = cm_(tmp().alloc((int64_t)it.m * k), it.m, k);
                gemm_c(Q[l], U, false, T, false, Z{1, 0}, false);         // Y = U V^* Omega
                RsBlk d{};
                d.yoff = Q[l].p - base;
                d.m = it.m / 3;
                d.k = k;
                ob[l] = d;
            }
            DeviceBuf d_ob;
            d_ob.alloc(ob.size() * sizeof(RsBlk));
            HM_HIP_CHECK(hipMemcpyAsync(d_ob.p, ob.data(), ob.size() * sizeof(RsBlk), hipMemcpyHostToDevice, st));
            launch_orth(d_ob.as<RsBlk>(), (int32_t)ob.size(), base, st, true);
            std::vector<DotItem> dz;
            for (size_t l = 0; l < live.size(); ++l) {
                const lu::RcItem &it = items[act[live[l]]];
                const int32_t k = s[live[l]];
                DMat U = cm_(it.U, it.m, it.K), V = cm_(it.V, it.n, it.K);
                DMat P = cm_(tmp().alloc((int64_t)it.K * k), it.K, k);
                gemm_c(P, adj(U), true, Q[l], false, Z{1, 0}, false);      // U^* Q
                Zm[l] = cm_(tmp().alloc((int64_t)it.n * k), it.n, k);
                gemm_c(Zm[l], V, false, P, false, Z{1, 0}, false);         // Z = V U^* Q = B^* Q
                dz.push_back({Zm[l].p, Zm[l].p, (int64_t)it.n * k});
            }
            const std::vector<double> nz = dots(dz);   // synchronizes: ob outlives its copy
            std::vector<size_t> next;
            for (size_t l = 0; l < live.size(); ++l) {
                const size_t a = live[l];
                lu::RcItem &it = items[act[a]];
                const int32_t k = s[a];
                if (nb[a] - nz[l] <= 0.25 * eps * eps * nb[a]) {
                    it.U = Q[l].p;
                    it.V = Zm[l].p;
                    it.K = k;
                    ++F.stats.n_sampled;
                } else if (2 * k < it.K && 2 * k <= kRsMaxK) {
                    s[a] = 2 * k;
                    next.push_back(a);
                }
            }
            live.swap(next);
        }
    }
    void copy(DMat dst, DMat src, Z alpha, bool cj, bool acc) {
        hipLaunchKernelGGL(lu_copy_kernel, dim3(grid_for((int64_t)dst.m * dst.n)), dim3(256), 0, st,
                           dst.p, dst.rs, dst.cs, src.p, src.rs, src.cs, dst.m, dst.n, alpha,
                           cj ? 1 : 0, acc ? 1 : 0);
        HM_HIP_CHECK(hipGetLastError());
    }
    void fill(DMat dst, Z diag) {
        hipLaunchKernelGGL(lu_fill_kernel, dim3(grid_for((int64_t)dst.m * dst.n)), dim3(256), 0, st,
                           dst.p, dst.rs, dst.cs, dst.m, dst.n, diag);
        HM_HIP_CHECK(hipGetLastError());
    }
    void getrf_inv(Z *D, Z *Linv, Z *Uinv, int32_t n) {
        hipLaunchKernelGGL(lu_getrf_kernel, dim3(1), dim3(1024), 0, st, D, n, F.d_flag.as<int32_t>());
        hipLaunchKernelGGL(lu_trinv_kernel, dim3((unsigned)ceil_div(n, 64), 2), dim3(64), 0, st, D, Linv,
                           Uinv, n);
        HM_HIP_CHECK(hipGetLastError());
    }
    // Every item through run_recompress / run_recompress_apply (offsets
    // counted from the first factor chunk; a zero row padding makes the U'
    // output plain column-major).
    void truncate(std::vector<lu::RcItem> &items, double eps_lu) {
        // The update matrices scale column c by s_c^-1/2 and s_c^-3/2: a
        // singular value at the rounding level of the core is noise, and
        // keeping it inflates the factors by orders of magnitude per
        // recompression until they overflow.  Tolerances below kEpsFloor act
        // as kEpsFloor.
        constexpr double kEpsFloor = 1e-13;
        const double eps = std::max(eps_lu, kEpsFloor);
        // |B|_F^2 - |Z|_F^2 certifies the sampled range only where eps^2 stays
        // well above the rounding of |B|_F^2
        if (eps >= 1e-6) range_finder(items, eps);
        Z *base = F.keep.base();
        std::vector<RcBlk> rc;
        int64_t goff = 0;
        for (const lu::RcItem &it : items) {
            RcBlk b;
            b.uoff = it.U - base;
            b.voff = it.V - base;
            b.goff = goff;
            b.m = it.m / 3;
            b.n = it.n / 3;
            b.r = it.K;
            b.rb = 0;
            goff += 8 * (int64_t)it.K * it.K + 2 * (int64_t)it.K;
            rc.push_back(b);
        }
        DeviceBuf d_rc, d_newrank, d_ou, d_ov;
        d_rc.alloc(rc.size() * sizeof(RcBlk));
        HM_HIP_CHECK(hipMemcpyAsync(d_rc.p, rc.data(), rc.size() * sizeof(RcBlk), hipMemcpyHostToDevice, st));
        d_newrank.alloc(rc.size() * sizeof(int32_t));
        Z *work = tmp().alloc(goff);
        run_recompress<double>(rc, d_rc.as<RcBlk>(), base, reinterpret_cast<double *>(work),
                               d_newrank.as<int32_t>(), eps, 0, st, false, rc.size() < 256);
        std::vector<int32_t> keep(rc.size());
        HM_HIP_CHECK(hipMemcpyAsync(keep.data(), d_newrank.p, keep.size() * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, st));
        HM_HIP_CHECK(hipStreamSynchronize(st));
        std::vector<int64_t> ou(rc.size(), 0), ov(rc.size(), 0);
        for (size_t i = 0; i < items.size(); ++i) {
            lu::RcItem &it = items[i];
            need(keep[i] >= 0 && keep[i] <= it.K, "H-LU: recompressed rank out of range");
            it.keep = keep[i];
            if (!it.keep) continue;
            it.Uout = keep_class_alloc(F, (int64_t)it.m * it.keep);
            it.Vrow = tmp().alloc((int64_t)it.n * lu::even(it.keep));
            ou[i] = it.Uout - base;
            ov[i] = it.Vrow - base;
        }
        d_ou.alloc(ou.size() * sizeof(int64_t));
        d_ov.alloc(ov.size() * sizeof(int64_t));
        HM_HIP_CHECK(hipMemcpyAsync(d_ou.p, ou.data(), ou.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
        HM_HIP_CHECK(hipMemcpyAsync(d_ov.p, ov.data(), ov.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
        run_recompress_apply<double>(rc, d_rc.as<RcBlk>(), base, reinterpret_cast<const double *>(work),
                                     d_ou.as<int64_t>(), d_ov.as<int64_t>(), d_newrank.as<int32_t>(),
                                     base, keep, F.d_zero_rowpad.as<int32_t>(), st, false);
        // the host vectors and buffers above outlive their copies and kernels
        HM_HIP_CHECK(hipStreamSynchronize(st));
    }
};

using GpuCore = lu::Core<GpuBackend>;

template <typename S>
void import_leaves(hm_lu &F, const hm_matrix *A, const std::vector<std::pair<int, int64_t>> &leaves,
                   const std::vector<int32_t> &leaf_block, hipStream_t st) {
    const cplx<S> *dense = A->dense.as<cplx<S>>();
    const cplx<S> *fac = A->factors<cplx<S>>();
    const int32_t *rp = A->d_rowpad.as<int32_t>();
    for (const auto &pr : leaves) {
        LuNode &X = F.nodes[pr.first];
        const int32_t b = leaf_block[pr.second];
        const Block &B = A->blocks[b];
        const int32_t slot = A->block_slot[b];
        if (B.kind == BLOCK_DENSE) {
            const DenseBlk &d = A->h_dblk[slot];
            X.kind = lu::FMT_F;
            X.D = F.keep.alloc((int64_t)X.m * X.n);
            hipLaunchKernelGGL(lu_import_dense_kernel<S>, dim3(grid_for((int64_t)X.m * X.n)), dim3(256),
                               0, st, dense + d.off, (int64_t)d.ld, rp, d.rb, d.m, 3 * d.n, X.D);
        } else {
            const LowRankBlk &L = A->h_lblk[slot];
            X.kind = lu::FMT_R;
            X.k = L.r;
            if (L.r > 0) {
                X.U = keep_class_alloc(F, (int64_t)X.m * L.r);
                X.W = keep_class_alloc(F, (int64_t)L.r * X.n);
                hipLaunchKernelGGL(lu_import_lr_kernel<S>,
                                   dim3(grid_for((int64_t)(X.m + X.n) * L.r)), dim3(256), 0, st,
                                   fac + L.uoff, (int64_t)L.ldu, fac + L.voff, (int64_t)L.ldv, rp,
                                   L.rb, L.m, L.n, L.r, X.U, X.W);
            }
        }
        HM_HIP_CHECK(hipGetLastError());
    }
}

// ---------------------------------------------- |A_H - A|_F and |A|_F
// One thread per point pair (p, q) of a block: the 3 x 3 kernel block (or
// the collocation operator's entry block, Coll) is evaluated in FP64 and
// compared with the stored one (dense tile, or the rows of U and V for a
// low-rank block).  Partial sums per workgroup.
struct FrobTask {
    int32_t slot, kind, p0, np;   // block (dense or low-rank slot), pairs p0 .. p0 + np
};

template <typename S, bool Coll>
__global__ void __launch_bounds__(256) frob_kernel(Geometry g, GreenParams<double> gp,
                                                   const FrobTask *__restrict__ tasks,
                                                   const DenseBlk *__restrict__ dblk,
                                                   const LowRankBlk *__restrict__ lblk,
                                                   const cplx<S> *__restrict__ dense,
                                                   const cplx<S> *__restrict__ fac,
                                                   const int32_t *__restrict__ rowpad,
                                                   double self_re, double self_im,
                                                   double *__restrict__ part) {
    const FrobTask tk = tasks[blockIdx.x];
    double sd = 0, sa = 0;
    for (int32_t e = threadIdx.x; e < tk.np; e += blockDim.x) {
        const int32_t pq = tk.p0 + e;
        int32_t rb, cb, m;
        if (tk.kind == 0) {
            rb = dblk[tk.slot].rb;
            cb = dblk[tk.slot].cb;
            m = dblk[tk.slot].m;
        } else {
            rb = lblk[tk.slot].rb;
            cb = lblk[tk.slot].cb;
            m = lblk[tk.slot].m;
        }
        const int32_t i = pq % m, j = pq / m;
        const int32_t pi = rb + i, pj = cb + j;
        cplx<double> K[9];
        if constexpr (Coll) {
            colloc_block<double>(g, gp, pi, pj, K);
        } else if (g.same && pi == pj) {
#pragma unroll
            for (int a = 0; a < 9; ++a) K[a] = {0, 0};
            K[0] = K[4] = K[8] = {self_re, self_im};
        } else {
            const double dx = g.x[0][pi] - g.y[0][pj];
            const double dy = g.x[1][pi] - g.y[1][pj];
            const double dz = g.x[2][pi] - g.y[2][pj];
            double nx = 0, ny = 0, nz = 0;
            if (gp.kind == 1) {
                nx = g.n[0][pj];
                ny = g.n[1][pj];
                nz = g.n[2][pj];
            }
            green_block<double>(gp, dx, dy, dz, nx, ny, nz, K);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int bcol = 0; bcol < 3; ++bcol) {
                cplx<double> h;
                if (tk.kind == 0) {
                    const DenseBlk &d = dblk[tk.slot];
                    h = cvt<double>(dense[d.off + (3 * (int64_t)j + bcol) * d.ld +
                                          padded_row(rowpad, rb, i, a)]);
                } else {
                    const LowRankBlk &L = lblk[tk.slot];
                    const cplx<S> *u = fac + L.uoff + padded_row(rowpad, rb, i, a);
                    const cplx<S> *v = fac + L.voff + (3 * (int64_t)j + bcol) * L.ldv;
                    h = {0, 0};
                    for (int c = 0; c < L.r; ++c) {
                        const cplx<double> uu = cvt<double>(u[(int64_t)c * L.ldu]);
                        const cplx<double> vv = cvt<double>(v[c]);
                        h = h + mulc(uu, vv);
                    }
                }
                const cplx<double> k = K[3 * a + bcol];
                sd += abs2(h - k);
                sa += abs2(k);
            }
    }
    __shared__ double red[2][4];
    sd = wave_sum(sd);
    sa = wave_sum(sa);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sd;
        red[1][threadIdx.x >> 6] = sa;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            a += red[0][w];
            b += red[1][w];
        }
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

__global__ void norm2_kernel(const Z *__restrict__ x, int64_t n, double *__restrict__ part) {
    double s = 0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        s += abs2(x[q]);
    __shared__ double red[4];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

double device_norm(const Z *x, int64_t n, hipStream_t st) {
    const unsigned nb = 1024;
    DeviceBuf part;
    part.alloc(nb * sizeof(double));
    hipLaunchKernelGGL(norm2_kernel, dim3(nb), dim3(256), 0, st, x, n, part.as<double>());
    HM_HIP_CHECK(hipGetLastError());
    std::vector<double> h(nb);
    HM_HIP_CHECK(hipMemcpyAsync(h.data(), part.p, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    HM_HIP_CHECK(hipStreamSynchronize(st));
    double s = 0;
    for (double v : h) s += v;
    return std::sqrt(s);
}

}  // namespace
}  // namespace hm

using namespace hm;

extern "C" hm_status hm_lu_factor(const hm_matrix *A, double eps_lu, void *stream, hm_lu **out) {
    HM_API_BEGIN
    need(A != nullptr && out != nullptr, "NULL argument");
    need(eps_lu >= 0.0, "eps_lu must be >= 0");
    if (A->plan_only) throw StatusError(HM_ERR_STATE, "matrix was built with plan_only");
    need(A->p.same != 0, "the H-LU needs a square operator on one point cloud (same = 1)");
    *out = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto F = std::make_unique<hm_lu>();
    F->eps = eps_lu;
    F->st = st;
    const ClusterTree &tr = A->rowtree();
    F->dofs = 3 * A->nx;
    // leaf blocks keyed by (row node, col node)
    std::vector<std::pair<int64_t, int32_t>> key;
    for (size_t b = 0; b < A->blocks.size(); ++b)
        key.push_back({(int64_t)A->blocks[b].row * tr.nodes() + A->blocks[b].col, (int32_t)b});
    std::sort(key.begin(), key.end());
    std::vector<int64_t> leaf_of(key.size());
    std::vector<int32_t> leaf_block(key.size());
    for (size_t i = 0; i < key.size(); ++i) {
        leaf_of[i] = key[i].first;
        leaf_block[i] = key[i].second;
    }
    std::vector<std::pair<int, int64_t>> leaves;
    const lu::TreeView tv{tr.begin.data(), tr.end.data(), tr.left.data(), tr.right.data(), tr.nodes()};
    lu::build_node(F->nodes, tv, leaf_of, 0, 0, leaves);
    need(leaves.size() == A->blocks.size(), "internal: block list and tree disagree");
    {
        std::vector<int32_t> zero(A->nx + 1, 0);
        F->d_zero_rowpad.alloc(zero.size() * sizeof(int32_t));
        HM_HIP_CHECK(hipMemcpyAsync(F->d_zero_rowpad.p, zero.data(), zero.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, st));
        F->d_perm.alloc(tr.perm.size() * sizeof(int32_t));
        HM_HIP_CHECK(hipMemcpyAsync(F->d_perm.p, tr.perm.data(), tr.perm.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, st));
        F->d_flag.alloc(sizeof(int32_t));
        HM_HIP_CHECK(hipMemsetAsync(F->d_flag.p, 0, sizeof(int32_t), st));
        HM_HIP_CHECK(hipStreamSynchronize(st));
    }
    if (A->p.prec == HM_C64)
        import_leaves<float>(*F, A, leaves, leaf_block, st);
    else
        import_leaves<double>(*F, A, leaves, leaf_block, st);
    HM_HIP_CHECK(hipStreamSynchronize(st));
    const auto t1 = std::chrono::steady_clock::now();
    // HM_LU_STREAMS (1 .. kLuStreams) sets the number of streams; the factors are
    // the same for every value
    int ns = kLuStreams;
    if (const char *env = std::getenv("HM_LU_STREAMS")) ns = std::max(1, std::min(kLuStreams, std::atoi(env)));
    // The extra streams, their stacks and the fork / join events live for this
    // call; on every exit path the streams are drained before anything is freed.
    struct Pool {
        std::vector<hipStream_t> streams;
        std::vector<hipEvent_t> events;
        std::vector<std::unique_ptr<Arena>> arenas;
        size_t bytes = 0;
        void drain() {
            for (hipStream_t s : streams) (void)hipStreamSynchronize(s);
            for (hipEvent_t e : events) (void)hipEventDestroy(e);
            events.clear();
            for (auto &a : arenas) bytes += a->total;
            arenas.clear();
            for (hipStream_t s : streams) (void)hipStreamDestroy(s);
            streams.clear();
        }
        ~Pool() { drain(); }
    } pool;
    GpuBackend be{*F, st};
    be.nstreams = ns;
    be.events = &pool.events;
    for (int k = 1; k < ns; ++k) {
        hipStream_t s = nullptr;
        HM_HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        pool.streams.push_back(s);
        pool.arenas.push_back(std::make_unique<Arena>(size_t(1) << 28));
        be.strm[k] = s;
        be.arena[k] = pool.arenas.back().get();
    }
    GpuCore c(be, F->nodes, eps_lu);
    c.hlu(0);
    need(be.cur == 0, "internal: unbalanced fork / join");
    int32_t zp = 0;
    HM_HIP_CHECK(hipMemcpyAsync(&zp, F->d_flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HM_HIP_CHECK(hipStreamSynchronize(st));
    pool.drain();
    if (zp) throw StatusError(HM_ERR_NOCONV, "zero pivot in a diagonal leaf (elimination without pivoting)");
    const auto t2 = std::chrono::steady_clock::now();
    c.tally(0);
    F->stats.t_import = std::chrono::duration<double>(t1 - t0).count();
    F->stats.t_factor = std::chrono::duration<double>(t2 - t1).count();
    F->stats.device_bytes = (int64_t)(F->keep.total + F->tmp.total + pool.bytes);
    F->stats.n_nodes = (int32_t)F->nodes.size();
    *out = F.release();
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_lu_solve(hm_lu *F, const void *b, void *x, int32_t nrhs, void *stream) {
    HM_API_BEGIN
    need(F != nullptr && b != nullptr && x != nullptr, "NULL argument");
    need(nrhs >= 1, "nrhs must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    GpuBackend be{*F, st};
    GpuCore c(be, F->nodes, F->eps);
    const auto mk = F->tmp.mark();
    DMat X = c.tmpmat((int32_t)F->dofs, nrhs, false);
    const int64_t tot = F->dofs * nrhs;
    hipLaunchKernelGGL(lu_gather_kernel, dim3(grid_for(tot)), dim3(256), 0, st,
                       static_cast<const Z *>(b), F->d_perm.as<int32_t>(), F->dofs, nrhs, X.p);
    HM_HIP_CHECK(hipGetLastError());
    c.lower_solve(0, X);
    c.upper_solve_left(0, X);
    hipLaunchKernelGGL(lu_scatter_kernel, dim3(grid_for(tot)), dim3(256), 0, st, X.p,
                       F->d_perm.as<int32_t>(), F->dofs, nrhs, static_cast<Z *>(x));
    HM_HIP_CHECK(hipGetLastError());
    F->tmp.release(mk);
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_lu_get_stats(const hm_lu *F, hm_lu_stats *s) {
    HM_API_BEGIN
    need(F != nullptr && s != nullptr, "NULL argument");
    *s = F->stats;
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_lu_export_dense(hm_lu *F, void *host_buf) {
    HM_API_BEGIN
    need(F != nullptr && host_buf != nullptr, "NULL argument");
    need(F->dofs <= 20000, "hm_lu_export_dense is for small problems (3N <= 20000)");
    hipStream_t st = F->st;
    GpuBackend be{*F, st};
    GpuCore c(be, F->nodes, F->eps);
    const auto mk = F->tmp.mark();
    DMat D = c.tmpmat((int32_t)F->dofs, (int32_t)F->dofs, false);
    c.densify(0, D);
    HM_HIP_CHECK(hipMemcpyAsync(host_buf, D.p, (size_t)F->dofs * F->dofs * sizeof(Z),
                                hipMemcpyDeviceToHost, st));
    HM_HIP_CHECK(hipStreamSynchronize(st));
    F->tmp.release(mk);
    return HM_OK;
    HM_API_END
}

extern "C" void hm_lu_destroy(hm_lu *F) { delete F; }

extern "C" hm_status hm_frob_error(const hm_matrix *A, void *stream, double *diff_fro,
                                   double *a_fro) {
    HM_API_BEGIN
    need(A != nullptr && diff_fro != nullptr && a_fro != nullptr, "NULL argument");
    if (A->plan_only) throw StatusError(HM_ERR_STATE, "matrix was built with plan_only");
    hipStream_t st = static_cast<hipStream_t>(stream);
    constexpr int32_t kPairs = 2048;
    std::vector<FrobTask> tasks;
    for (size_t i = 0; i < A->h_dblk.size(); ++i) {
        const int32_t np = A->h_dblk[i].m * A->h_dblk[i].n;
        for (int32_t p0 = 0; p0 < np; p0 += kPairs) tasks.push_back({(int32_t)i, 0, p0, std::min(kPairs, np - p0)});
    }
    for (size_t i = 0; i < A->h_lblk.size(); ++i) {
        const int32_t np = A->h_lblk[i].m * A->h_lblk[i].n;
        for (int32_t p0 = 0; p0 < np; p0 += kPairs) tasks.push_back({(int32_t)i, 1, p0, std::min(kPairs, np - p0)});
    }
    DeviceBuf d_tasks, d_d, d_l, part;
    auto up = [&](DeviceBuf &buf, const void *src, size_t bytes) {
        buf.alloc(std::max<size_t>(bytes, 16));
        if (bytes) HM_HIP_CHECK(hipMemcpyAsync(buf.p, src, bytes, hipMemcpyHostToDevice, st));
    };
    up(d_tasks, tasks.data(), tasks.size() * sizeof(FrobTask));
    up(d_d, A->h_dblk.data(), A->h_dblk.size() * sizeof(DenseBlk));
    up(d_l, A->h_lblk.data(), A->h_lblk.size() * sizeof(LowRankBlk));
    part.alloc(std::max<size_t>(tasks.size(), 1) * 2 * sizeof(double));
    const GreenParams<double> gp =
        make_green_params<double>(A->p.kernel, A->p.omega, A->p.lambda, A->p.mu, A->p.rho);
    if (!tasks.empty()) {
        const bool coll = !A->h_tri.empty();
        const auto kf = coll ? frob_kernel<float, true> : frob_kernel<float, false>;
        const auto kd = coll ? frob_kernel<double, true> : frob_kernel<double, false>;
        if (A->p.prec == HM_C64)
            hipLaunchKernelGGL(kf, dim3((unsigned)tasks.size()), dim3(256), 0, st,
                               A->geometry(), gp, d_tasks.as<FrobTask>(), d_d.as<DenseBlk>(),
                               d_l.as<LowRankBlk>(), A->dense.as<cplx<float>>(),
                               A->factors<cplx<float>>(), A->d_rowpad.as<int32_t>(), A->p.self_re,
                               A->p.self_im, part.as<double>());
        else
            hipLaunchKernelGGL(kd, dim3((unsigned)tasks.size()), dim3(256), 0, st,
                               A->geometry(), gp, d_tasks.as<FrobTask>(), d_d.as<DenseBlk>(),
                               d_l.as<LowRankBlk>(), A->dense.as<cplx<double>>(),
                               A->factors<cplx<double>>(), A->d_rowpad.as<int32_t>(), A->p.self_re,
                               A->p.self_im, part.as<double>());
        HM_HIP_CHECK(hipGetLastError());
    }
    std::vector<double> h(2 * tasks.size());
    if (!h.empty())
        HM_HIP_CHECK(hipMemcpyAsync(h.data(), part.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HM_HIP_CHECK(hipStreamSynchronize(st));
    double sd = 0, sa = 0;
    for (size_t i = 0; i < tasks.size(); ++i) {
        sd += h[2 * i];
        sa += h[2 * i + 1];
    }
    *diff_fro = std::sqrt(sd);
    *a_fro = std::sqrt(sa);
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_lu_estimate(const hm_matrix *A, const void *b, const void *x0,
                                    double delta_h, void *stream, hm_lu_estimate_t *est) {
    HM_API_BEGIN
    need(A != nullptr && b != nullptr && x0 != nullptr && est != nullptr, "NULL argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = 3 * A->nx;
    DeviceBuf r;
    r.alloc(n * sizeof(Z));
    const hm_status s = hm_residual(A, b, x0, r.p, 1, stream);
    if (s != HM_OK) return s;
    est->delta = device_norm(r.as<Z>(), n, st);
    est->b_norm = device_norm(static_cast<const Z *>(b), n, st);
    est->x0_norm = device_norm(static_cast<const Z *>(x0), n, st);
    est->delta_h = delta_h;
    est->estimate = (est->delta + delta_h * est->x0_norm) / est->b_norm;
    return HM_OK;
    HM_API_END
}
