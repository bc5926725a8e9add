// Internal structures of the hmat library shared by the API layer and the
// kernel translation units.
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"
#include "green.hpp"
#include "tree.hpp"

namespace hm {

// Dense near-field tile: rows rb..rb+m (row cluster order), cols cb..cb+n,
// stored column-major (3m x 3n) at `off` complex elements into the dense slab.
// Storage layout shared by dense tiles and U factors: the rows of a row
// cluster are the concatenation of its leaves' row segments (3 per point),
// each padded with one zero row when odd, so every leaf segment starts at an
// even row (16-byte aligned complex64 pairs).  rowpad(P) below is that
// padding count before cluster position P.
struct DenseBlk {
    int64_t off;
    int32_t rb, m, cb, n;
    int32_t ld, pad;     // ld = padded row count of the tile (even)
};

// Low-rank block U V^*: U (3m x r) column-major at uoff, V (3n x r) row-major
// at voff, t-vector slot at toff (r entries per right-hand side).
struct LowRankBlk {
    int64_t uoff, voff, toff;
    int32_t rb, m, cb, n, r;
    int32_t ldu;         // padded row count of U (even)
    int32_t ldv;         // row stride of the row-major V: r rounded up to even
    int32_t pad;
};

// Work item of a leaf row cluster: kind 0 = dense block index, 1 = low-rank
// block index; rowoff = first row of the leaf inside the block (points).
struct Task {
    int32_t kind, idx, rowoff, pad;
};

// Projection work item: one wave computes the contribution of rows
// row0..row0+nrows of a block to t for columns col0..col0+63; single-chunk
// items write t directly (slot < 0), the others write partial sums to
// tpart[slot * 64 + c] which a reduction pass adds up.
struct ProjTask {
    int32_t blk, col0, row0, nrows, slot, pad;
};

// Reduction of the partial projections of one (block, col0) group.
struct ProjReduce {
    int32_t blk, col0, slot0, nslots;
};

constexpr int32_t kProjRows = 512;
// Admissible blocks with at least this many points (m + n) run their ACA in
// the split form (each step spread over many workgroups) and come first in an
// ACA launch.
constexpr int kAcaBigPoints = 1500;

// Multi-RHS (matrix-core) plan.  Accumulation: one wave per 16 rows of a
// leaf row cluster's segment.  Projection: one wave per (low-rank block, 16
// rows of T = V^* X, chunk k0..k0+klen of the contraction over 3n); slot < 0
// writes T directly, otherwise a partial summed by an MrProjReduce.
struct MrAccItem {
    int32_t leaf, row0, pad0, pad1;
};
struct MrProjItem {
    int32_t blk, j0, k0, klen, slot, pad;
};
struct MrProjReduce {
    int32_t blk, j0, slot0, nslots;
};
constexpr int32_t kMrPanel = 64;    // right-hand sides per panel
constexpr int32_t kMrChunk = 768;   // contraction chunk of a projection item
constexpr int32_t kMrMinCols = 8;   // panels are used from this many right-hand sides on

struct LeafRow {
    int32_t rb, m, tbeg, tend;
};

// ACA work description for one admissible block.
struct AcaBlk {
    int64_t uoff, voff;   // scratch factor offsets (complex elements)
    int64_t foff;         // offset of the used-flag bytes (m + n)
    int32_t rb, m, cb, n;
    int32_t budget;       // column budget
    // r0 > 0: the block resumes a run that stopped at its budget; its first
    // r0 factor columns and its used flags are already in place, and the
    // run's step count, fallbacks, next row pivot, the column count of its
    // last term whose stopping test is still open (split ACA) and
    // ||B_k||_F^2 follow.
    int32_t r0;
    int32_t steps0, fallbacks0, ih0, pend0;
    double norm0;
};

struct AcaOut {
    int32_t rank;
    int32_t status;       // 0 converged, 1 budget exhausted, 2 full rank
    int32_t fallbacks;
    int32_t steps;
    double norm2;         // recursive ||B_k||_F^2
    int32_t ih;           // next row pivot (meaningful for status 1)
    int32_t pend;         // columns of the last term whose stopping test is open (status 1)
};

// Randomized range finder (rsvd.hip) for admissible blocks whose 3x3
// sub-blocks are all singular.  RsIn: one block on the host (input rb, m, cb,
// n; output k, factor offsets and the FP64 norms); RsBlk: its device
// descriptor for one attempt; RsTask: 64 rows of a product.
constexpr int32_t kRsMaxK = 256;   // largest number of samples per block
struct RsIn {
    int32_t rb, m, cb, n;
    int64_t aoff = 0;          // dense block in the batch's dense scratch
    int32_t k = 0, buf = -1;   // accepted samples; attempt buffer holding them
    int64_t uoff = 0, voff = 0;   // factors in the returned scratch (ACA layout)
    double norm2 = 0, range_err2 = 0;   // |A|_F^2 and |A - Q Q^* A|_F^2
};
struct RsBlk {
    int64_t aoff, omoff, yoff, boff, uoff, voff;
    int32_t m, n, k, pad;
};
struct RsTask {
    int32_t blk, row0, pad0, pad1;
};


// In place Q = orth(Y) for every descriptor (Y at base + yoff, 3m x k
// column-major, k <= kRsMaxK): classical Gram-Schmidt with one
// reorthogonalisation, dependent columns set to zero; one workgroup each
// (1024 threads when wide, for calls with few descriptors, else 256).
void launch_orth(const RsBlk *d_blk, int32_t nblk, cplx<double> *base, hipStream_t st,
                 bool wide = false);

// Recompression work description.
struct RcBlk {
    int64_t uoff, voff;   // ACA factors (scratch slab)
    int64_t goff;         // r x r FP64 work matrices offset (complex doubles)
    int32_t m, n, r, rb;  // rb: first row point (cluster order) for the padded U layout
};

// Owning device buffer.  Memory comes from the library's device cache:
// buffers of at least 32 MiB are kept on release and handed out again for
// requests of up to that size (and at least half of it), because freeing and
// re-allocating tens of GB costs the driver up to seconds; release
// synchronizes the device first, as hipFree would.  hm_release_cache()
// returns the cached memory to the driver.
struct DeviceBuf {
    void *p = nullptr;
    size_t bytes = 0;   // capacity
    int dev = 0;
    DeviceBuf() = default;
    DeviceBuf(const DeviceBuf &) = delete;
    DeviceBuf &operator=(const DeviceBuf &) = delete;
    ~DeviceBuf() { reset(); }
    void reset();
    void alloc(size_t b);
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
};

// HIP event without timing, destroyed with its scope.
struct ScopedEvent {
    hipEvent_t e = nullptr;
    ScopedEvent() {
        const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r != hipSuccess) throw HipError(std::string("hipEventCreateWithFlags: ") +
                                                hipGetErrorString(r), r);
    }
    ScopedEvent(const ScopedEvent &) = delete;
    ScopedEvent &operator=(const ScopedEvent &) = delete;
    ~ScopedEvent() {
        if (e) (void)hipEventDestroy(e);
    }
};

size_t elem_bytes(int prec);  // bytes of one complex element

}  // namespace hm

struct hm_matrix {
    hm_params p{};
    int64_t nx = 0, ny = 0;
    bool plan_only = false;
    hm::ClusterTree tx, ty;             // ty unused when same
    std::vector<hm::Block> blocks;
    std::vector<int32_t> rank, rank_aca;  // per block (-1 for dense)
    std::vector<int64_t> off_a, off_v;    // per block storage offsets
    hm_stats stats{};

    // P1 collocation operator (Section 4): elements in original vertex
    // numbers and the quadrature orders; empty for a point operator
    std::vector<int32_t> h_tri;
    int32_t q_reg = 0, q_sing = 0;
    hm::DeviceBuf d_mesh;     // int32: elements, incidence pointers, incidence (cluster order)
    hm::DeviceBuf d_rule;     // float64 (s, t, w) triples: regular, then singular rule

    // device data
    hm::DeviceBuf geo;        // 9 SoA float64 arrays (x, y, n)
    hm::DeviceBuf perm_x, perm_y;
    hm::DeviceBuf dense;      // dense slab
    // U and V factors, one buffer per assembly chunk; every LowRankBlk offset
    // counts complex elements from lr_base (the first chunk's buffer), so the
    // offsets of later chunks may be negative or span the gap between buffers
    std::vector<std::unique_ptr<hm::DeviceBuf>> lowrank;
    void *lr_base = nullptr;
    template <typename T>
    T *factors() const { return static_cast<T *>(lr_base); }
    hm::DeviceBuf d_dblk, d_lblk, d_tasks, d_leaves, d_ptasks, d_preduce, tpart;
    int32_t n_dblk = 0, n_lblk = 0, n_leaves = 0, n_ptasks = 0, n_preduce = 0;
    int32_t max_leaf = 1;     // largest leaf row cluster (points)
    int32_t acc_waves = 8;    // waves per workgroup of the 1-RHS accumulation (4, 8, 16)
    int32_t proj_rows = hm::kProjRows;   // row chunk of the 1-RHS projection items
    int32_t proj_slots = 0;   // partial-sum slots (64 entries each) of the projection plan
    hm::DeviceBuf d_rowpad;   // int32[nx + 1]: padding rows before each position
    std::vector<int32_t> rowpad;
    int64_t t_len = 0;        // sum of ranks
    std::vector<hm::DenseBlk> h_dblk;
    std::vector<hm::LowRankBlk> h_lblk;
    std::vector<int32_t> block_slot;  // block id -> index into h_dblk / h_lblk

    // lazily sized work buffers for matvec
    hm::DeviceBuf ws_xc, ws_t, ws_y;

    // multi-RHS plan (complex64 operators) and its workspaces, allocated on
    // first use
    hm::DeviceBuf d_mracc, d_mrproj, d_mrred;
    int32_t n_mracc = 0, n_mrproj = 0, n_mrred = 0, mr_nslots = 0;
    mutable hm::DeviceBuf ws_x64, ws_t64, ws_tp64;

    // captured matvec (p.matvec_graph): the executable graph, the key it was
    // captured for, and the private stream used for capturing
    mutable hipGraphExec_t g_exec = nullptr;
    mutable const void *g_x = nullptr;
    mutable void *g_y = nullptr;
    mutable int32_t g_nrhs = 0;
    mutable hipStream_t g_stream = nullptr;

    hm_matrix() = default;
    hm_matrix(const hm_matrix &) = delete;
    hm_matrix &operator=(const hm_matrix &) = delete;
    ~hm_matrix() {
        if (g_exec) (void)hipGraphExecDestroy(g_exec);
        if (g_stream) (void)hipStreamDestroy(g_stream);
    }

    const hm::ClusterTree &rowtree() const { return tx; }
    const hm::ClusterTree &coltree() const { return p.same ? tx : ty; }
    hm::Geometry geometry() const;
};

namespace hm {

// ---- kernel launchers (implemented in the .hip files) ----
template <typename R>
void launch_nearfield(const Geometry &g, const GreenParams<R> &gp, const DenseBlk *d_blk,
                      int32_t nblk, cplx<R> *slab, R self_re, R self_im, int32_t *d_err,
                      hipStream_t st, bool unbatched);

// y = A x for one right-hand side column (c of nrhs), S = storage real, A = accumulation
template <typename S, typename A>
void launch_matvec_col(const hm_matrix *M, const void *x, int64_t ldx, int32_t col, void *y,
                       int64_t ldy, const double *b, hipStream_t st);

// Allocates the multi-RHS panel workspaces on first use.
void ensure_mrhs_workspace(const hm_matrix *M);

// Y[:, col0 .. col0+ncols) = A X[:, col0 .. col0+ncols), ncols <= 64,
// complex64 operators only; ev (optional) receives 4 event records.
void launch_matvec_mrhs(const hm_matrix *M, const void *x, int64_t ldx, int32_t col0,
                        int32_t ncols, void *y, int64_t ldy, hipStream_t st, hipEvent_t *ev);

// Extra streams per device (which = 0, 1) for independent work of one build:
// default priority, non-blocking, created on first use, kept until exit.
hipStream_t side_stream(int which);

// Rank-model features of the admissible blocks (block-list order) and a
// forward pass of the model on them.
void rank_features(const hm_matrix *M, std::vector<float> &feats, std::vector<int64_t> &ids);
void rank_predict(const float *w_host, const std::vector<float> &feats, std::vector<float> &pred,
                  hipStream_t st);

template <typename S>
void profile_matvec_col(const hm_matrix *M, const void *x, void *y, hipStream_t st, double *ms3);

template <typename R>
void run_aca(const Geometry &g, const GreenParams<R> &gp, const std::vector<AcaBlk> &blk,
             AcaBlk *d_blk, cplx<R> *scratchU, uint8_t *flags, AcaOut *d_out, double eps,
             double tau_piv, int32_t max_budget, hipStream_t st, bool unbatched,
             hipStream_t aux);

// Randomized range finder for the blocks blk (see rsvd.hip); factors receives
// the ACA-layout factor scratch (U = Q: 3m x k, V = B^*: 3n x k).
template <typename R>
void run_rsvd(const Geometry &g, const GreenParams<R> &gp, std::vector<RsIn> &blk, double eps,
              int k0, uint64_t seed, std::unique_ptr<DeviceBuf> &factors, hipStream_t st);

// Recompression of ACA factors in place into compact output.
template <typename R>
void run_recompress(const std::vector<RcBlk> &blk, RcBlk *d_blk, const cplx<R> *acaslab,
                    double *work, int32_t *d_newrank, double eps, int32_t rmax, hipStream_t st,
                    bool unbatched, bool wide_small = false);

template <typename R>
void run_recompress_apply(const std::vector<RcBlk> &blk, RcBlk *d_blk, const cplx<R> *acaslab,
                          const double *work, const int64_t *d_outu, const int64_t *d_outv,
                          const int32_t *d_newrank, cplx<R> *out, const std::vector<int32_t> &keep,
                          const int32_t *d_rowpad, hipStream_t st, bool unbatched);

// Padded row of (local point p, component a) in a block whose row cluster
// starts at cluster position rb.
__host__ __device__ inline int64_t padded_row(const int32_t *rowpad, int32_t rb, int32_t p, int a) {
    return 3 * (int64_t)p + a + (rowpad[rb + p] - rowpad[rb]);
}
__host__ __device__ inline int32_t padded_rows(const int32_t *rowpad, int32_t rb, int32_t m) {
    return 3 * m + (rowpad[rb + m] - rowpad[rb]);
}
__host__ __device__ inline int32_t even_up(int32_t v) { return v + (v & 1); }

}  // namespace hm

// Exception-to-status translation around every C entry point.
#define HM_API_BEGIN try {
#define HM_API_END                                               \
    }                                                            \
    catch (const hm::StatusError &e) {                           \
        hm::set_error(e.msg);                                    \
        return e.status;                                         \
    }                                                            \
    catch (const hm::HipError &e) {                              \
        hm::set_error(e.msg);                                    \
        (void)hipGetLastError();                                 \
        return HM_ERR_HIP;                                       \
    }                                                            \
    catch (const std::bad_alloc &) {                             \
        hm::set_error("host allocation failed");                 \
        return HM_ERR_ALLOC;                                     \
    }                                                            \
    catch (const std::exception &e) {                            \
        hm::set_error(e.what());                                 \
        return HM_ERR_ARG;                                       \
    }
