// C ABI entry points: argument validation, host planning, device assembly
// orchestration, matvec dispatch and exports.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <atomic>
#include <future>
#include <mutex>
#include <numeric>
#include <string>

#include "internal.hpp"

namespace {
thread_local std::string g_last_error;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

namespace hm {

void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

struct CachedBlock {
    void *p;
    size_t bytes;
    int dev;
};
std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;
std::atomic<int64_t> g_live_bytes{0};   // device bytes held by live DeviceBufs
constexpr size_t kCacheMin = size_t(32) << 20;

// Smallest cached block on `dev` holding b bytes and at most twice b.
bool cache_take(size_t b, int dev, void **p, size_t *cap) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    size_t best = SIZE_MAX;
    for (size_t i = 0; i < g_cache.size(); ++i) {
        const CachedBlock &c = g_cache[i];
        if (c.dev == dev && c.bytes >= b && c.bytes <= 2 * b &&
            (best == SIZE_MAX || c.bytes < g_cache[best].bytes))
            best = i;
    }
    if (best == SIZE_MAX) return false;
    *p = g_cache[best].p;
    *cap = g_cache[best].bytes;
    g_cache.erase(g_cache.begin() + (std::ptrdiff_t)best);
    return true;
}

// Bytes held in the cache for `dev`.
size_t cache_bytes(int dev) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    size_t s = 0;
    for (const CachedBlock &c : g_cache)
        if (c.dev == dev) s += c.bytes;
    return s;
}

void cache_release_all() {
    std::vector<CachedBlock> blocks;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        blocks.swap(g_cache);
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (const CachedBlock &c : blocks) {
        (void)hipSetDevice(c.dev);
        (void)hipFree(c.p);
    }
    (void)hipSetDevice(cur);
}

}  // namespace

hipStream_t side_stream(int which) {
    static std::mutex mu;
    static hipStream_t streams[2][64] = {};
    int dev = 0;
    HM_HIP_CHECK(hipGetDevice(&dev));
    if (which < 0 || which > 1 || dev < 0 || dev >= 64)
        throw StatusError(HM_ERR_HIP, "side stream index out of range");
    std::lock_guard<std::mutex> lk(mu);
    if (!streams[which][dev])
        HM_HIP_CHECK(hipStreamCreateWithFlags(&streams[which][dev], hipStreamNonBlocking));
    return streams[which][dev];
}

void DeviceBuf::reset() {
    if (!p) return;
    g_live_bytes -= (int64_t)bytes;
    if (bytes >= kCacheMin) {
        // as hipFree would: no queued work may still use the memory
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(dev);
        (void)hipDeviceSynchronize();
        (void)hipSetDevice(cur);
        std::lock_guard<std::mutex> lk(g_cache_mu);
        g_cache.push_back({p, bytes, dev});
    } else {
        (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
}

void DeviceBuf::alloc(size_t b) {
    reset();
    if (b == 0) return;
    // Failure injection for tests: with HM_FAULT_ALLOC=k the k-th device
    // allocation of this thread fails, counted from the last time the
    // variable's value changed.
    const char *inj = std::getenv("HM_FAULT_ALLOC");
    if (inj) {
        static thread_local long counter = 0;
        static thread_local std::string seen;
        if (seen != inj) {
            seen = inj;
            counter = 0;
        }
        if (++counter == std::atol(inj)) throw StatusError(HM_ERR_ALLOC, "injected allocation failure");
    }
    HM_HIP_CHECK(hipGetDevice(&dev));
    if (b >= kCacheMin / 2 && cache_take(b, dev, &p, &bytes)) {
        g_live_bytes += (int64_t)bytes;
        return;
    }
    hipError_t e = hipMalloc(&p, b);
    if (e == hipErrorOutOfMemory) {
        // give the cached blocks back and try once more
        (void)hipGetLastError();
        cache_release_all();
        e = hipMalloc(&p, b);
    }
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        throw StatusError(HM_ERR_ALLOC, "hipMalloc of " + std::to_string(b) + " bytes failed: " +
                                            hipGetErrorString(e) + " (the library holds " +
                                            std::to_string(g_live_bytes.load()) +
                                            " bytes in live buffers)");
    }
    bytes = b;
    g_live_bytes += (int64_t)b;
}

size_t elem_bytes(int prec) { return prec == HM_C64 ? 8 : 16; }

template <typename T>
static void upload(DeviceBuf &buf, const std::vector<T> &v, hipStream_t st) {
    buf.alloc(std::max<size_t>(v.size(), 1) * sizeof(T));
    if (!v.empty()) {
        // The source is pageable host memory that may be freed right after
        // this call returns, so the copy completes before returning.
        HM_HIP_CHECK(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
        HM_HIP_CHECK(hipStreamSynchronize(st));
    }
}

// Copies the leading r columns of ACA factors into the final slab: U to the
// padded column-major layout, V transposed to row-major with an even stride.
template <typename R>
__global__ void copy_factors_kernel(const RcBlk *__restrict__ blks, const cplx<R> *__restrict__ src,
                                    const int64_t *__restrict__ outu,
                                    const int64_t *__restrict__ outv, cplx<R> *__restrict__ dst,
                                    const int32_t *__restrict__ rowpad) {
    const RcBlk b = blks[blockIdx.y];
    const int64_t rows_u = 3 * (int64_t)b.m, rows_v = 3 * (int64_t)b.n;
    const int64_t nu = rows_u * b.r, nv = rows_v * b.r;
    const int64_t ldu = padded_rows(rowpad, b.rb, b.m), ldv = even_up(b.r);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nu + nv;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (k < nu) {
            const int64_t row = k % rows_u, c = k / rows_u;
            dst[outu[blockIdx.y] + c * ldu +
                padded_row(rowpad, b.rb, (int32_t)(row / 3), (int)(row % 3))] = src[b.uoff + k];
        } else {
            const int64_t q = k - nu;
            const int64_t row = q % rows_v, c = q / rows_v;
            dst[outv[blockIdx.y] + row * ldv + c] = src[b.voff + q];
        }
    }
}

}  // namespace hm

using namespace hm;

hm::Geometry hm_matrix::geometry() const {
    Geometry g{};
    const double *base = geo.as<double>();
    for (int a = 0; a < 3; ++a) g.x[a] = base + a * nx;
    if (p.same) {
        for (int a = 0; a < 3; ++a) g.y[a] = g.x[a];
    } else {
        for (int a = 0; a < 3; ++a) g.y[a] = base + 3 * nx + a * ny;
    }
    const double *nb = base + 3 * nx + (p.same ? 0 : 3 * ny);
    for (int a = 0; a < 3; ++a) g.n[a] = (p.kernel == HM_KERNEL_T) ? nb + a * ny : nullptr;
    g.same = p.same;
    if (!h_tri.empty() && d_mesh.p) {
        const int64_t ne = (int64_t)h_tri.size() / 3;
        const int32_t *mb = d_mesh.as<int32_t>();
        g.mesh.tri = mb;
        g.mesh.inc_ptr = mb + 3 * ne;
        g.mesh.inc = mb + 3 * ne + nx + 1;
        g.mesh.rule = d_rule.as<double>();
        g.mesh.nreg = q_reg * q_reg;
        g.mesh.nsing = q_sing * q_sing;
    }
    return g;
}

static void require(bool ok, const std::string &msg) {
    if (!ok) throw StatusError(HM_ERR_ARG, msg);
}

// 1-RHS projection items: every (block, 64 columns of V) split into row
// chunks of `chunk` rows; multi-chunk groups get a reduction item.  Largest
// items first.
static void build_project_plan(hm_matrix *M, int32_t chunk, hipStream_t st) {
    std::vector<ProjTask> ptasks;
    std::vector<ProjReduce> preduce;
    int32_t nslots = 0;
    for (int32_t i = 0; i < M->n_lblk; ++i) {
        const int32_t rows = 3 * M->h_lblk[i].n;
        const int32_t nch = (int32_t)ceil_div(rows, chunk);
        for (int32_t c0 = 0; c0 < M->h_lblk[i].r; c0 += 64) {
            if (nch == 1) {
                ptasks.push_back({i, c0, 0, rows, -1, 0});
                continue;
            }
            preduce.push_back({i, c0, nslots, nch});
            for (int32_t ch = 0; ch < nch; ++ch)
                ptasks.push_back({i, c0, ch * chunk, std::min(chunk, rows - ch * chunk), nslots++, 0});
        }
    }
    std::stable_sort(ptasks.begin(), ptasks.end(), [&](const ProjTask &a, const ProjTask &b) {
        return (int64_t)a.nrows * std::min(64, M->h_lblk[a.blk].r - a.col0) >
               (int64_t)b.nrows * std::min(64, M->h_lblk[b.blk].r - b.col0);
    });
    M->n_ptasks = (int32_t)ptasks.size();
    M->n_preduce = (int32_t)preduce.size();
    M->proj_rows = chunk;
    M->proj_slots = nslots;
    upload(M->d_ptasks, ptasks, st);
    upload(M->d_preduce, preduce, st);
    M->tpart.alloc(std::max<int64_t>(nslots, 1) * 64 * sizeof(cplx<double>));
}

extern "C" hm_status hm_params_default(hm_params *p) {
    if (!p) return HM_ERR_ARG;
    std::memset(p, 0, sizeof(*p));
    p->kernel = HM_KERNEL_U;
    p->prec = HM_C128;
    p->omega = 1.0;
    p->lambda = 2.0;
    p->mu = 1.0;
    p->rho = 1.0;
    p->eta = 3.0;
    p->eps = 1e-4;
    p->leaf = 32;
    p->same = 1;
    p->recompress = 1;
    p->rsvd = 1;
    return HM_OK;
}

extern "C" const char *hm_last_error(void) { return g_last_error.c_str(); }

namespace {

std::vector<double> fetch_points(const double *ptr, int64_t n, bool on_host, const char *what) {
    std::vector<double> h(3 * n);
    if (on_host) {
        std::memcpy(h.data(), ptr, h.size() * sizeof(double));
    } else {
        HM_HIP_CHECK(hipMemcpy(h.data(), ptr, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    }
    for (double v : h) require(std::isfinite(v), std::string("non-finite value in ") + what);
    return h;
}

// Leaves of the subtree rooted at v (pre-order numbering: subtree = v..).
void leaves_under(const ClusterTree &t, int32_t v, std::vector<int32_t> &out) {
    std::vector<int32_t> st{v};
    while (!st.empty()) {
        const int32_t u = st.back();
        st.pop_back();
        if (t.is_leaf(u)) {
            out.push_back(u);
        } else {
            st.push_back(t.right[u]);
            st.push_back(t.left[u]);
        }
    }
}

template <typename R>
void assemble_device(hm_matrix *M, const std::vector<double> &X, const std::vector<double> &Y,
                     const std::vector<double> &Nrm, hipStream_t st);

// Gauss-Legendre nodes and weights on [0, 1]: the roots of the Legendre
// polynomial P_q by Newton's method from x = cos(pi (i + 3/4) / (q + 1/2)),
// weights 2 / ((1 - x^2) P_q'(x)^2), both mapped from [-1, 1].
void gauss_legendre01(int q, std::vector<double> &x, std::vector<double> &w) {
    x.assign(q, 0.0);
    w.assign(q, 0.0);
    for (int i = 0; i < (q + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (q + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = q * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute P_q' at the converged root
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = q * (z * p1 - p0) / (z * z - 1.0);
        }
        const double wt = 1.0 / ((1.0 - z * z) * dp * dp);   // half of 2 / (...)
        x[i] = 0.5 * (1.0 - z);
        x[q - 1 - i] = 0.5 * (1.0 + z);
        w[i] = w[q - 1 - i] = wt;
    }
}

// Collapsed product rule: (s, t, w_s w_t s) for the q x q Gauss-Legendre points.
void collapsed_rule(int q, std::vector<double> &out) {
    std::vector<double> g, w;
    gauss_legendre01(q, g, w);
    for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b) {
            out.push_back(g[a]);
            out.push_back(g[b]);
            out.push_back(w[a] * w[b] * g[a]);
        }
}

// Elements (cluster positions), the elements around each vertex and the two
// quadrature rules of a collocation operator, uploaded for Colloc.
void upload_mesh(hm_matrix *M, hipStream_t st) {
    const ClusterTree &tx = M->rowtree();
    const int64_t nc = M->nx, ne = (int64_t)M->h_tri.size() / 3;
    std::vector<int32_t> pos(nc);
    for (int64_t k = 0; k < nc; ++k) pos[tx.perm[k]] = (int32_t)k;
    std::vector<int32_t> buf(3 * ne + nc + 1 + 3 * ne, 0);
    int32_t *tri = buf.data(), *ptr = tri + 3 * ne, *inc = ptr + nc + 1;
    for (int64_t q = 0; q < 3 * ne; ++q) tri[q] = pos[M->h_tri[q]];
    for (int64_t q = 0; q < 3 * ne; ++q) ++ptr[tri[q] + 1];
    for (int64_t v = 0; v < nc; ++v) ptr[v + 1] += ptr[v];
    std::vector<int32_t> fill(ptr, ptr + nc);
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) inc[fill[tri[3 * e + k]]++] = (int32_t)(4 * e + k);
    upload(M->d_mesh, buf, st);
    std::vector<double> rule;
    collapsed_rule(M->q_reg, rule);
    collapsed_rule(M->q_sing, rule);
    upload(M->d_rule, rule, st);
}

hm_status build_impl(const double *x, int64_t nx, const double *y, int64_t ny,
                     const double *normals, const hm_params *p, void *stream, hm_matrix **out,
                     const std::vector<int32_t> *tri, int32_t q_reg, int32_t q_sing);

}  // namespace

extern "C" hm_status hm_build(const double *x, int64_t nx, const double *y, int64_t ny,
                              const double *normals, const hm_params *p, void *stream,
                              hm_matrix **out) {
    return build_impl(x, nx, y, ny, normals, p, stream, out, nullptr, 0, 0);
}

extern "C" hm_status hm_build_colloc(const double *nodes, int64_t nc, const int32_t *tri, int64_t ne,
                                     int32_t q_reg, int32_t q_sing, const hm_params *p,
                                     void *stream, hm_matrix **out) {
    if (out) *out = nullptr;
    hm::set_error("");
    HM_API_BEGIN
    require(p != nullptr, "params is NULL");
    require(p->kernel == HM_KERNEL_U,
            "collocation operators are built for the single-layer (U) kernel only");
    require(nodes != nullptr && nc >= 3, "nodes must be non-NULL with nc >= 3");
    require(tri != nullptr && ne >= 1 && ne < (int64_t)1 << 28, "tri must be non-NULL with ne >= 1");
    require(q_reg >= 1 && q_reg <= 32 && q_sing >= 1 && q_sing <= 32,
            "quadrature orders must lie in 1 .. 32");
    std::vector<int32_t> t(3 * ne);
    if (p->points_on_host)
        std::memcpy(t.data(), tri, t.size() * sizeof(int32_t));
    else
        HM_HIP_CHECK(hipMemcpy(t.data(), tri, t.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<int32_t> deg(nc, 0);
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t a = t[3 * e], b = t[3 * e + 1], c = t[3 * e + 2];
        require(a >= 0 && a < nc && b >= 0 && b < nc && c >= 0 && c < nc,
                "element vertex out of range");
        require(a != b && b != c && a != c, "element with a repeated vertex");
        ++deg[a], ++deg[b], ++deg[c];
    }
    for (int64_t v = 0; v < nc; ++v) require(deg[v] > 0, "a vertex belongs to no element");
    hm_params q = *p;
    q.same = 1;
    q.self_re = q.self_im = 0.0;
    q.rsvd = 0;
    return build_impl(nodes, nc, nullptr, nc, nullptr, &q, stream, out, &t, q_reg, q_sing);
    HM_API_END
}

namespace {

hm_status build_impl(const double *x, int64_t nx, const double *y, int64_t ny,
                     const double *normals, const hm_params *p, void *stream, hm_matrix **out,
                     const std::vector<int32_t> *tri, int32_t q_reg, int32_t q_sing) {
    if (out) *out = nullptr;
    hm::set_error("");
    HM_API_BEGIN
    require(out != nullptr, "out is NULL");
    require(p != nullptr, "params is NULL");
    require(x != nullptr && nx >= 1, "x must be non-NULL with nx >= 1");
    require(p->kernel == HM_KERNEL_U || p->kernel == HM_KERNEL_T, "unknown kernel");
    require(p->prec == HM_C128 || p->prec == HM_C64, "unknown precision");
    require(std::isfinite(p->omega) && p->omega >= 0, "omega must be finite and >= 0");
    require(std::isfinite(p->mu) && p->mu > 0, "mu must be > 0");
    require(std::isfinite(p->rho) && p->rho > 0, "rho must be > 0");
    require(std::isfinite(p->lambda) && p->lambda + 2 * p->mu > 0, "lambda + 2 mu must be > 0");
    require(std::isfinite(p->eta) && p->eta >= 0, "eta must be >= 0");
    require(std::isfinite(p->eps) && p->eps > 0 && p->eps < 1, "eps must lie in (0, 1)");
    require(p->leaf >= 1, "leaf must be >= 1");
    require(nx < (int64_t)1 << 30, "too many points");
    if (p->same) {
        ny = nx;
    } else {
        require(y != nullptr && ny >= 1, "y must be non-NULL with ny >= 1 when same == 0");
        require(ny < (int64_t)1 << 30, "too many points");
    }
    if (p->kernel == HM_KERNEL_T) require(normals != nullptr, "normals are required for T");
    const bool on_host = p->points_on_host != 0;
    auto M = std::make_unique<hm_matrix>();
    M->p = *p;
    M->nx = nx;
    M->ny = ny;
    M->plan_only = p->plan_only != 0;
    if (tri) {
        M->h_tri = *tri;
        M->q_reg = q_reg;
        M->q_sing = q_sing;
    }
    const double t0 = now_s();
    std::vector<double> X = fetch_points(x, nx, on_host, "x");
    std::vector<double> Y, Nrm;
    if (!p->same) Y = fetch_points(y, ny, on_host, "y");
    if (p->kernel == HM_KERNEL_T) Nrm = fetch_points(normals, ny, on_host, "normals");
    M->tx = build_cluster_tree(X.data(), nx, p->leaf);
    if (!p->same) M->ty = build_cluster_tree(Y.data(), ny, p->leaf);
    M->blocks = build_block_tree(M->tx, M->coltree(), p->eta);
    const double t1 = now_s();
    const ClusterTree &tx = M->rowtree(), &ty = M->coltree();
    const int64_t nb = (int64_t)M->blocks.size();
    M->rank.assign(nb, -1);
    M->rank_aca.assign(nb, -1);
    hm_stats &S = M->stats;
    S.nx = nx;
    S.ny = ny;
    S.nodes_x = tx.nodes();
    S.nodes_y = ty.nodes();
    auto count_leaves = [](const ClusterTree &t) {
        int32_t c = 0;
        for (int32_t v = 0; v < t.nodes(); ++v) c += t.is_leaf(v);
        return c;
    };
    S.leaves_x = count_leaves(tx);
    S.leaves_y = count_leaves(ty);
    S.levels_x = 1 + *std::max_element(tx.depth.begin(), tx.depth.end());
    S.levels_y = 1 + *std::max_element(ty.depth.begin(), ty.depth.end());
    S.n_blocks = nb;
    std::vector<int32_t> crow(tx.nodes(), 0), ccol(ty.nodes(), 0);
    for (const auto &b : M->blocks) {
        (b.kind == BLOCK_DENSE ? S.n_dense : S.n_lowrank)++;
        crow[b.row]++;
        ccol[b.col]++;
    }
    S.c_sp = std::max(*std::max_element(crow.begin(), crow.end()),
                      *std::max_element(ccol.begin(), ccol.end()));
    S.prec = p->prec;
    S.t_tree = t1 - t0;
    if (!M->plan_only) {
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (p->prec == HM_C64)
            assemble_device<float>(M.get(), X, Y, Nrm, st);
        else
            assemble_device<double>(M.get(), X, Y, Nrm, st);
    }
    S.t_total = now_s() - t0;
    *out = M.release();
    return HM_OK;
    HM_API_END
}

template <typename R>
void assemble_device(hm_matrix *M, const std::vector<double> &X, const std::vector<double> &Y,
                     const std::vector<double> &Nrm, hipStream_t st) {
    const hm_params &p = M->p;
    const ClusterTree &tx = M->rowtree(), &ty = M->coltree();
    hm_stats &S = M->stats;
    const int64_t nx = M->nx, ny = M->ny;
    double t = now_s();
    // ---- geometry in cluster order, SoA float64 ------------------------
    {
        const size_t n_geo = 3 * nx + (p.same ? 0 : 3 * ny) + (p.kernel == HM_KERNEL_T ? 3 * ny : 0);
        std::vector<double> h(n_geo);
        for (int a = 0; a < 3; ++a)
            for (int64_t k = 0; k < nx; ++k) h[a * nx + k] = X[3 * (int64_t)tx.perm[k] + a];
        size_t off = 3 * nx;
        if (!p.same) {
            for (int a = 0; a < 3; ++a)
                for (int64_t k = 0; k < ny; ++k) h[off + a * ny + k] = Y[3 * (int64_t)ty.perm[k] + a];
            off += 3 * ny;
        }
        if (p.kernel == HM_KERNEL_T)
            for (int a = 0; a < 3; ++a)
                for (int64_t k = 0; k < ny; ++k) h[off + a * ny + k] = Nrm[3 * (int64_t)ty.perm[k] + a];
        upload(M->geo, h, st);
        upload(M->perm_x, tx.perm, st);
        if (!p.same) upload(M->perm_y, ty.perm, st);
        if (!M->h_tri.empty()) upload_mesh(M, st);
    }
    const Geometry g = M->geometry();
    const GreenParams<R> gp = make_green_params<R>(p.kernel, p.omega, p.lambda, p.mu, p.rho);
    HM_HIP_CHECK(hipStreamSynchronize(st));
    S.t_upload = now_s() - t;
    t = now_s();
    const int64_t nb = (int64_t)M->blocks.size();
    M->block_slot.assign(nb, -1);
    M->off_a.assign(nb, -1);
    M->off_v.assign(nb, -1);
    // ---- padded row layout: every leaf segment (3 rows per point) is padded
    // with zero rows to a multiple of kSegRows, so that every segment of every
    // column starts on a kSegRows-row boundary: 128-byte lines in complex128
    // (8 rows), 16-byte row pairs in complex64 (2 rows; whole 128-byte lines,
    // 16 rows, were measured there too: no faster, about 10% more storage).
    constexpr int32_t kSegRows = sizeof(R) == 8 ? 8 : 2;
    M->rowpad.assign(nx + 1, 0);
    {
        int32_t acc = 0;
        for (int32_t v = 0; v < tx.nodes(); ++v) {
            if (!tx.is_leaf(v)) continue;   // pre-order visits leaves in position order
            for (int32_t q = tx.begin[v]; q < tx.end[v]; ++q) M->rowpad[q] = acc;
            acc += (kSegRows - (3 * tx.size(v)) % kSegRows) % kSegRows;
        }
        M->rowpad[nx] = acc;
    }
    upload(M->d_rowpad, M->rowpad, st);
    const int32_t *rowpad = M->rowpad.data();
    // ---- dense near-field tiles ------------------------------------------
    int64_t dense_entries = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const Block &B = M->blocks[b];
        if (B.kind != BLOCK_DENSE) continue;
        DenseBlk d;
        d.off = dense_entries;
        d.rb = tx.begin[B.row];
        d.m = tx.size(B.row);
        d.cb = ty.begin[B.col];
        d.n = ty.size(B.col);
        d.ld = padded_rows(rowpad, d.rb, d.m);
        d.pad = 0;
        M->block_slot[b] = (int32_t)M->h_dblk.size();
        M->off_a[b] = d.off;
        M->h_dblk.push_back(d);
        dense_entries += (int64_t)d.ld * 3 * d.n;
    }
    M->n_dblk = (int32_t)M->h_dblk.size();
    // +2 elements: paired 16-byte loads may touch one element past the last tile
    M->dense.alloc((dense_entries + 2) * sizeof(cplx<R>));
    HM_HIP_CHECK(hipMemsetAsync(M->dense.p, 0, (dense_entries + 2) * sizeof(cplx<R>), st));
    upload(M->d_dblk, M->h_dblk, st);
    DeviceBuf derr;
    derr.alloc(sizeof(int32_t));
    HM_HIP_CHECK(hipMemsetAsync(derr.p, 0, sizeof(int32_t), st));
    launch_nearfield<R>(g, gp, M->d_dblk.as<DenseBlk>(), M->n_dblk, M->dense.as<cplx<R>>(),
                        R(p.self_re), R(p.self_im), derr.as<int32_t>(), st, p.unbatched != 0);
    int32_t nerr = 0;
    HM_HIP_CHECK(hipMemcpyAsync(&nerr, derr.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HM_HIP_CHECK(hipStreamSynchronize(st));
    if (nerr) throw StatusError(HM_ERR_SINGULAR, std::to_string(nerr) +
                                                     " coincident point pairs outside self blocks");
    S.dense_entries = dense_entries;
    S.t_nearfield = now_s() - t;
    t = now_s();
    // ---- vector ACA on admissible blocks -----------------------------------
    std::vector<int64_t> lr_ids;
    for (int64_t b = 0; b < nb; ++b)
        if (M->blocks[b].kind == BLOCK_LOWRANK) lr_ids.push_back(b);
    const int64_t nlr = (int64_t)lr_ids.size();
    double tau_piv = p.tau_piv > 0 ? p.tau_piv : (sizeof(R) == 4 ? 1e-4 : 1e-8);
    const int32_t def_budget = p.rank_budget > 0 ? p.rank_budget : 96;
    std::vector<int32_t> budget(nlr), lm(nlr), ln(nlr);
    for (int64_t k = 0; k < nlr; ++k) {
        const Block &B = M->blocks[lr_ids[k]];
        lm[k] = tx.size(B.row);
        ln[k] = ty.size(B.col);
        const int32_t full = 3 * std::min(lm[k], ln[k]);
        // Size-aware first budget (a rank prediction, when given, replaces it).
        const int32_t big = std::max(lm[k], ln[k]);
        int32_t b0 = def_budget;
        if (p.rank_budget <= 0) b0 = big < 400 ? 96 : (big < 1000 ? 192 : 288);
        budget[k] = std::min(full, std::max(b0, 3));
        budget[k] = std::max(3, budget[k] - budget[k] % 3);
    }
    // A rank model replaces the size rule: first budget = predicted rank
    // * 1.25 + 6, rounded up to a multiple of 3.
    std::vector<uint8_t> from_model(nlr, 0);
    if (p.rank_model != nullptr && nlr > 0) {
        std::vector<float> feats, pred;
        std::vector<int64_t> ids;
        rank_features(M, feats, ids);
        rank_predict(p.rank_model, feats, pred, st);
        for (int64_t k = 0; k < nlr; ++k) {
            const double rh = 3.0 * (std::exp2(std::min(20.0, (double)pred[k])) - 1.0);
            int32_t b0 = (int32_t)std::ceil(1.25 * std::max(0.0, rh) + 6.0);
            b0 += (3 - b0 % 3) % 3;
            budget[k] = std::max(3, std::min(b0, 3 * std::min(lm[k], ln[k])));
            from_model[k] = 1;
        }
    }
    int32_t overflow = 0, fallbacks = 0, capped = 0, hits = 0;
    // The one-workgroup ACA kernel keeps the pivot row (3 x budget, compute
    // type) and the V Gram column (budget x 3, complex FP64) in LDS: the
    // budget is capped so that both fit in 60 KiB (852 columns in complex64,
    // 639 in complex128).  The split form would allow three times as many
    // (only its pivot row is in LDS), but the blocks that reach the cap are
    // ones whose ACA stagnates: on the 254,546-point T sphere at kappa_s = 84
    // they ran on to 2,559 columns for a recompressed rank of 515 and took
    // 85 s, so the split form keeps the same cap.  A block still unconverged
    // at the cap keeps its capped-rank approximation (hm_stats.n_capped).
    const int32_t budget_cap =
        (int32_t)((60 * 1024) / (3 * (sizeof(cplx<R>) + sizeof(cplx<double>)))) / 3 * 3;
    auto cap_of = [&](int64_t) { return budget_cap; };
    for (int64_t k = 0; k < nlr; ++k) budget[k] = std::min(budget[k], cap_of(k));
    // Longest first: ACA step k costs O(k (m + n)), a block about budget^2 (m + n).
    auto lpt = [&](int64_t a, int64_t b) {
        return (int64_t)(lm[a] + ln[a]) * budget[a] * budget[a] >
               (int64_t)(lm[b] + ln[b]) * budget[b] * budget[b];
    };
    std::vector<int64_t> order(nlr);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), lpt);
    // Blocks for the randomized range finder (params.rsvd): T kernel, both
    // clusters in one coordinate plane x_a = c (flat boxes at the same c) and
    // every column normal +-e_a, so that every 3x3 sub-block has the planar
    // pattern of Section 2.3 and is singular.
    std::vector<int64_t> rs_order;
    if (p.rsvd && p.kernel == HM_KERNEL_T && nlr > 0) {
        std::vector<uint8_t> nmask(ty.nodes(), 0);
        for (int32_t v = 0; v < ty.nodes(); ++v) {
            uint8_t mk = 7;
            for (int32_t q = ty.begin[v]; q < ty.end[v] && mk; ++q) {
                const double *nv = &Nrm[3 * (int64_t)ty.perm[q]];
                for (int a = 0; a < 3; ++a)
                    if (std::fabs(nv[a]) != 1.0 || nv[(a + 1) % 3] != 0.0 || nv[(a + 2) % 3] != 0.0)
                        mk &= (uint8_t)~(1u << a);
            }
            nmask[v] = mk;
        }
        std::vector<int64_t> rest;
        for (int64_t k : order) {
            const Block &B = M->blocks[lr_ids[k]];
            bool planar = false;
            for (int a = 0; a < 3 && !planar; ++a) {
                const double c = tx.lo[3 * B.row + a];
                planar = ((nmask[B.col] >> a) & 1) && tx.hi[3 * B.row + a] == c &&
                         ty.lo[3 * B.col + a] == c && ty.hi[3 * B.col + a] == c;
            }
            (planar ? rs_order : rest).push_back(k);
        }
        order.swap(rest);
    }
    // The admissible blocks are processed in chunks whose first-pass factor
    // scratch stays about under a cap: a chunk's ACA, recompression and final
    // factors are done, and its scratch released, before the next chunk
    // starts.  The default cap is 40% of the device memory free when the
    // chunk starts (the library's cached blocks count as free), so that the
    // factors kept from earlier chunks shrink later ones.  The blocks not yet
    // compressed are dealt round-robin in the longest-first order, so that
    // every chunk has the same mix of long and short blocks.
    auto chunk_cap = [&]() -> int64_t {
        if (p.aca_scratch_mb > 0) return (int64_t)p.aca_scratch_mb << 20;
        size_t fr = 0, tot = 0;
        int dev = 0;
        HM_HIP_CHECK(hipMemGetInfo(&fr, &tot));
        HM_HIP_CHECK(hipGetDevice(&dev));
        return std::max<int64_t>(int64_t(1) << 30, (int64_t)((fr + cache_bytes(dev)) / 5 * 2));
    };
    auto first_need = [&](int64_t k) {
        return 3 * (int64_t)(lm[k] + ln[k]) * budget[k] * (int64_t)sizeof(cplx<R>);
    };
    std::vector<int32_t> aca_rank(nlr, 0), final_rank(nlr, 0);
    std::vector<int64_t> aca_u(nlr), aca_v(nlr), fu(nlr), fv(nlr);
    // A block that uses up its budget continues later from where it stopped:
    // its factor columns and used flags wait in a holding buffer, its loop
    // state here.  The continued run takes the same steps as one run with the
    // larger budget would.
    struct Resume {
        int32_t r = 0, steps = 0, fallbacks = 0, ih = 0, pend = 0;
        double norm2 = 0.0;
        const cplx<R> *u = nullptr, *v = nullptr;
        const uint8_t *f = nullptr;
    };
    std::vector<Resume> resume(nlr);
    std::vector<uint8_t> reran(nlr, 0);   // the first budget did not suffice
    // Holding buffers, released once every block they hold has continued
    // (used_gen catches up with the generation the block was held in).
    struct Held {
        std::unique_ptr<DeviceBuf> fac, flg;
        std::vector<std::pair<int64_t, int32_t>> blocks;   // (block, generation)
    };
    std::vector<Held> holding;
    std::vector<int32_t> hold_gen(nlr, 0), used_gen(nlr, 0);
    int32_t n_chunks_done = 0;
    int64_t lr_entries = 0, t_len = 0;
    double t_aca = 0.0, t_rc = 0.0;
    S.aca_scratch_bytes = 0;
    // With several chunks, the blocks that outgrow their first budget are
    // collected from every chunk and compressed together in one last chunk,
    // so that their long re-runs and large recompressions overlap each other
    // instead of ending every chunk.
    // The deferred blocks form the final phase, chunked by the same cap (their
    // budgets have grown); blocks that outgrow a budget there continue at once.
    std::vector<int64_t> deferred;
    std::vector<int64_t> remaining = order;
    bool chunked = false, last = false;
    int32_t n_rsvd = 0;
    for (;;) {
        // randomized range finder batches first: dense blocks plus FP64 samples
        // under half the chunk cap
        std::vector<int64_t> rs_members;
        if (!rs_order.empty()) {
            const int64_t cap = std::max<int64_t>(int64_t(1) << 30, chunk_cap() / 2);
            int64_t used = 0;
            size_t q = 0;
            for (; q < rs_order.size(); ++q) {
                const int64_t k = rs_order[q];
                const int64_t need = 9 * (int64_t)lm[k] * ln[k] * (int64_t)sizeof(cplx<R>) +
                                     3 * (int64_t)(lm[k] + ln[k]) * 2 * kRsMaxK * 16;
                if (q > 0 && used + need > cap) break;
                used += need;
                rs_members.push_back(k);
            }
            rs_order.erase(rs_order.begin(), rs_order.begin() + (std::ptrdiff_t)q);
        } else if (remaining.empty()) {
            if (last || deferred.empty()) break;
            last = true;
            remaining.swap(deferred);
            std::stable_sort(remaining.begin(), remaining.end(), lpt);
        }
        std::vector<int64_t> members;
        const bool rs_chunk = !rs_members.empty();
        if (rs_chunk) {
            members.swap(rs_members);
        } else {
            int64_t need = 0;
            for (int64_t k : remaining) need += first_need(k);
            const int64_t stride =
                std::max<int64_t>(1, std::min<int64_t>((int64_t)remaining.size(),
                                                       ceil_div(need, chunk_cap())));
            chunked = chunked || stride > 1;
            std::vector<int64_t> rest;
            for (size_t q = 0; q < remaining.size(); ++q)
                (q % stride == 0 ? members : rest).push_back(remaining[q]);
            remaining.swap(rest);
        }
        const bool defer = !last && chunked;
        double tc = now_s();
        // ---- vector ACA passes of the chunk, pipelined with recompression ------
        // Pass 0 runs every block of the chunk; blocks that use up their budget
        // run again with a doubled budget in the next pass.  Pass p + 1 runs on
        // its own stream while pass p is recompressed.
        std::vector<std::unique_ptr<DeviceBuf>> pass_scratch;
        std::vector<std::vector<int64_t>> pass_members;
        struct AcaLaunch {
            std::vector<int64_t> todo;
            std::vector<AcaBlk> ab;
            std::unique_ptr<DeviceBuf> scratch, flags, d_ab, d_out;
            hipStream_t s = nullptr;
            int64_t scratch_bytes = 0;
        };
        // launch() may run on a worker thread beside the main thread's
        // launch(): it writes only its own AcaLaunch and reads per-block state
        // of its own blocks; shared totals are added by the main thread.
        auto launch = [&](std::vector<int64_t> todo, hipStream_t s) {
            AcaLaunch L;
            // blocks with many points first (they run in the split form), each
            // group longest first
            std::stable_sort(todo.begin(), todo.end(), [&](int64_t a, int64_t b) {
                const bool ba = lm[a] + ln[a] >= kAcaBigPoints, bb = lm[b] + ln[b] >= kAcaBigPoints;
                return ba != bb ? ba : lpt(a, b);
            });
            L.ab.resize(todo.size());
            int64_t fac = 0, flg = 0;
            int32_t maxb = 3;
            for (size_t q = 0; q < todo.size(); ++q) {
                const int64_t k = todo[q];
                const Block &B = M->blocks[lr_ids[k]];
                AcaBlk &a = L.ab[q];
                a.rb = tx.begin[B.row];
                a.m = lm[k];
                a.cb = ty.begin[B.col];
                a.n = ln[k];
                a.budget = budget[k];
                a.uoff = fac;
                fac += 3 * (int64_t)a.m * a.budget;
                a.voff = fac;
                fac += 3 * (int64_t)a.n * a.budget;
                a.foff = flg;
                flg += a.m + a.n;
                // LDS of the one-workgroup kernel (split blocks size their own)
                if (a.m + a.n < kAcaBigPoints) maxb = std::max(maxb, a.budget);
                const Resume &rs = resume[k];
                if (rs.r > 0) {
                    a.r0 = rs.r;
                    a.steps0 = rs.steps;
                    a.fallbacks0 = rs.fallbacks;
                    a.ih0 = rs.ih;
                    a.pend0 = rs.pend;
                    a.norm0 = rs.norm2;
                }
            }
            L.scratch_bytes = fac * (int64_t)sizeof(cplx<R>);
            L.scratch = std::make_unique<DeviceBuf>();
            L.flags = std::make_unique<DeviceBuf>();
            L.d_ab = std::make_unique<DeviceBuf>();
            L.d_out = std::make_unique<DeviceBuf>();
            L.scratch->alloc(std::max<int64_t>(fac, 1) * sizeof(cplx<R>));
            L.flags->alloc(std::max<int64_t>(flg, 1));
            // resumed blocks: earlier columns and flags into the new buffers
            for (size_t q = 0; q < todo.size(); ++q) {
                const AcaBlk &a = L.ab[q];
                if (a.r0 <= 0) continue;
                const Resume &rs = resume[todo[q]];
                HM_HIP_CHECK(hipMemcpyAsync(L.scratch->template as<cplx<R>>() + a.uoff, rs.u,
                                            3 * (size_t)a.m * a.r0 * sizeof(cplx<R>),
                                            hipMemcpyDeviceToDevice, s));
                HM_HIP_CHECK(hipMemcpyAsync(L.scratch->template as<cplx<R>>() + a.voff, rs.v,
                                            3 * (size_t)a.n * a.r0 * sizeof(cplx<R>),
                                            hipMemcpyDeviceToDevice, s));
                used_gen[todo[q]] = hold_gen[todo[q]];
                HM_HIP_CHECK(hipMemcpyAsync(L.flags->template as<uint8_t>() + a.foff, rs.f,
                                            (size_t)(a.m + a.n), hipMemcpyDeviceToDevice, s));
            }
            upload(*L.d_ab, L.ab, s);
            L.d_out->alloc(L.ab.size() * sizeof(AcaOut));
            run_aca<R>(g, gp, L.ab, static_cast<AcaBlk *>(L.d_ab->p),
                       static_cast<cplx<R> *>(L.scratch->p), static_cast<uint8_t *>(L.flags->p),
                       static_cast<AcaOut *>(L.d_out->p), p.eps, tau_piv, maxb, s,
                       p.unbatched != 0, s == st && !p.unbatched ? side_stream(0) : nullptr);
            L.todo.swap(todo);
            L.s = s;
            return L;
        };
        // Waits for a launched pass and records it; returns the blocks to re-run.
        auto finish = [&](AcaLaunch &L) {
            std::vector<AcaOut> res(L.ab.size());
            HM_HIP_CHECK(hipMemcpyAsync(res.data(), L.d_out->p, res.size() * sizeof(AcaOut),
                                        hipMemcpyDeviceToHost, L.s));
            HM_HIP_CHECK(hipStreamSynchronize(L.s));
            std::vector<int64_t> next;
            const int32_t pass = (int32_t)pass_scratch.size();
            pass_members.emplace_back();
            // blocks that continue later keep their columns and flags
            {
                int64_t hf = 0, hb = 0;
                for (size_t q = 0; q < L.todo.size(); ++q)
                    if (res[q].status == 1 && budget[L.todo[q]] < cap_of(L.todo[q])) {
                        hf += 3 * (int64_t)(L.ab[q].m + L.ab[q].n) * res[q].rank;
                        hb += L.ab[q].m + L.ab[q].n;
                    }
                if (hb > 0) {
                    Held hd;
                    auto hfac = std::make_unique<DeviceBuf>(), hflg = std::make_unique<DeviceBuf>();
                    hfac->alloc(std::max<int64_t>(hf, 1) * sizeof(cplx<R>));
                    hflg->alloc(hb);
                    int64_t of = 0, ob = 0;
                    for (size_t q = 0; q < L.todo.size(); ++q) {
                        const int64_t k = L.todo[q];
                        if (!(res[q].status == 1 && budget[k] < cap_of(k))) continue;
                        const AcaBlk &a = L.ab[q];
                        const int32_t rk = res[q].rank;
                        cplx<R> *hu = hfac->template as<cplx<R>>() + of;
                        cplx<R> *hv = hu + 3 * (int64_t)a.m * rk;
                        uint8_t *hg = hflg->template as<uint8_t>() + ob;
                        HM_HIP_CHECK(hipMemcpyAsync(hu, L.scratch->template as<cplx<R>>() + a.uoff,
                                                    3 * (size_t)a.m * rk * sizeof(cplx<R>),
                                                    hipMemcpyDeviceToDevice, L.s));
                        HM_HIP_CHECK(hipMemcpyAsync(hv, L.scratch->template as<cplx<R>>() + a.voff,
                                                    3 * (size_t)a.n * rk * sizeof(cplx<R>),
                                                    hipMemcpyDeviceToDevice, L.s));
                        HM_HIP_CHECK(hipMemcpyAsync(hg, L.flags->template as<uint8_t>() + a.foff,
                                                    (size_t)(a.m + a.n), hipMemcpyDeviceToDevice,
                                                    L.s));
                        resume[k] = {rk, res[q].steps, res[q].fallbacks, res[q].ih, res[q].pend,
                                     res[q].norm2, hu, hv, hg};
                        hd.blocks.emplace_back(k, ++hold_gen[k]);
                        of += 3 * (int64_t)(a.m + a.n) * rk;
                        ob += a.m + a.n;
                    }
                    HM_HIP_CHECK(hipStreamSynchronize(L.s));
                    hd.fac = std::move(hfac);
                    hd.flg = std::move(hflg);
                    holding.push_back(std::move(hd));
                }
            }
            for (size_t q = 0; q < L.todo.size(); ++q) {
                const int64_t k = L.todo[q];
                if (res[q].status == 1 && budget[k] < cap_of(k)) {
                    ++overflow;
                    reran[k] = 1;
                    budget[k] = std::min({3 * std::min(lm[k], ln[k]), 2 * budget[k], cap_of(k)});
                    next.push_back(k);
                    continue;
                }
                if (res[q].status == 1) ++capped;
                if (!reran[k] && from_model[k]) ++hits;
                aca_rank[k] = res[q].rank;
                aca_u[k] = L.ab[q].uoff;
                aca_v[k] = L.ab[q].voff;
                fallbacks += res[q].fallbacks;
                pass_members[pass].push_back(k);
            }
            pass_scratch.push_back(std::move(L.scratch));
            L.flags.reset();
            L.d_ab.reset();
            L.d_out.reset();
            return next;
        };
        // Recompression of pass ps on the build stream, and the final factors
        // of its blocks.  The blocks go in groups whose FP64 recompression
        // work (8 r^2 + 2r complex doubles per block) stays under a cap; each
        // group's factors are written to a buffer of their own at once, and
        // the pass's ACA scratch is released at the end.  Every block's factor
        // offsets count from the first buffer (M->lr_base), the base pointer
        // of the matvec kernels; allocations are 256-byte aligned, so the
        // distance between two buffers is a whole (for complex64, even)
        // number of elements.
        auto compress_emit = [&](size_t ps) {
            const auto &mem = pass_members[ps];
            const int64_t work_cap =
                std::max<int64_t>(int64_t(1) << 30, chunk_cap() / 4) / (int64_t)sizeof(cplx<double>);
            size_t q0 = 0;
            while (q0 < mem.size()) {
                std::vector<RcBlk> rc;
                int64_t goff = 0;
                size_t q1 = q0;
                for (; q1 < mem.size(); ++q1) {
                    const int64_t k = mem[q1];
                    const int64_t wk = 8 * (int64_t)aca_rank[k] * aca_rank[k] + 2 * (int64_t)aca_rank[k];
                    if (q1 > q0 && goff + wk > work_cap) break;
                    RcBlk c;
                    c.uoff = aca_u[k];
                    c.voff = aca_v[k];
                    c.m = lm[k];
                    c.rb = tx.begin[M->blocks[lr_ids[k]].row];
                    c.n = ln[k];
                    c.r = aca_rank[k];
                    c.goff = goff;
                    goff += wk;
                    rc.push_back(c);
                }
                DeviceBuf d_rc, d_newrank, work;
                upload(d_rc, rc, st);
                d_newrank.alloc(rc.size() * sizeof(int32_t));
                if (p.recompress) {
                    work.alloc(std::max<int64_t>(goff, 1) * sizeof(cplx<double>));
                    run_recompress<R>(rc, d_rc.as<RcBlk>(), pass_scratch[ps]->as<cplx<R>>(),
                                      work.as<double>(), d_newrank.as<int32_t>(), p.eps, 0, st,
                                      p.unbatched != 0);
                    std::vector<int32_t> nr(rc.size());
                    HM_HIP_CHECK(hipMemcpyAsync(nr.data(), d_newrank.p, nr.size() * sizeof(int32_t),
                                                hipMemcpyDeviceToHost, st));
                    HM_HIP_CHECK(hipStreamSynchronize(st));
                    for (size_t q = q0; q < q1; ++q) final_rank[mem[q]] = nr[q - q0];
                } else {
                    for (size_t q = q0; q < q1; ++q) final_rank[mem[q]] = aca_rank[mem[q]];
                }
                // this group's final factors
                int64_t len = 0;
                std::vector<int64_t> ou(rc.size()), ov(rc.size());
                std::vector<int32_t> kp(rc.size());
                for (size_t q = q0; q < q1; ++q) {
                    const int64_t k = mem[q];
                    const Block &B = M->blocks[lr_ids[k]];
                    kp[q - q0] = final_rank[k];
                    ou[q - q0] = len;
                    len += (int64_t)padded_rows(rowpad, tx.begin[B.row], lm[k]) * final_rank[k];
                    ov[q - q0] = len;
                    len += 3 * (int64_t)ln[k] * even_up(final_rank[k]);
                    len += (kSegRows - len % kSegRows) % kSegRows;   // next U on a segment boundary
                }
                auto out = std::make_unique<DeviceBuf>();
                out->alloc((len + 2) * sizeof(cplx<R>));
                HM_HIP_CHECK(hipMemsetAsync(out->p, 0, (len + 2) * sizeof(cplx<R>), st));
                if (!M->lr_base) M->lr_base = out->p;
                const std::ptrdiff_t gap =
                    static_cast<const char *>(out->p) - static_cast<const char *>(M->lr_base);
                if (gap % (std::ptrdiff_t)(kSegRows * sizeof(cplx<R>)) != 0)
                    throw HipError("factor buffer misaligned against the first one",
                                   hipErrorInvalidValue);
                const int64_t delta = (int64_t)(gap / (std::ptrdiff_t)sizeof(cplx<R>));
                DeviceBuf d_ou, d_ov;
                upload(d_ou, ou, st);
                upload(d_ov, ov, st);
                if (p.recompress) {
                    run_recompress_apply<R>(rc, d_rc.as<RcBlk>(), pass_scratch[ps]->as<cplx<R>>(),
                                            work.as<double>(), d_ou.as<int64_t>(),
                                            d_ov.as<int64_t>(), d_newrank.as<int32_t>(),
                                            out->as<cplx<R>>(), kp, M->d_rowpad.as<int32_t>(), st,
                                            p.unbatched != 0);
                } else {
                    hipLaunchKernelGGL(copy_factors_kernel<R>, dim3(64, (unsigned)rc.size()),
                                       dim3(256), 0, st, d_rc.as<RcBlk>(),
                                       pass_scratch[ps]->as<cplx<R>>(), d_ou.as<int64_t>(),
                                       d_ov.as<int64_t>(), out->as<cplx<R>>(),
                                       M->d_rowpad.as<int32_t>());
                    HM_HIP_CHECK(hipGetLastError());
                }
                HM_HIP_CHECK(hipStreamSynchronize(st));
                for (size_t q = q0; q < q1; ++q) {
                    fu[mem[q]] = delta + ou[q - q0];
                    fv[mem[q]] = delta + ov[q - q0];
                }
                M->lowrank.push_back(std::move(out));
                lr_entries += len;
                q0 = q1;
            }
            pass_scratch[ps].reset();
        };
        hipStream_t aca_side = p.unbatched ? st : side_stream(1);
        if (rs_chunk) {
            // randomized range finder, then the usual recompression to eps
            std::vector<RsIn> in(members.size());
            for (size_t q = 0; q < members.size(); ++q) {
                const Block &B = M->blocks[lr_ids[members[q]]];
                in[q].rb = tx.begin[B.row];
                in[q].m = lm[members[q]];
                in[q].cb = ty.begin[B.col];
                in[q].n = ln[members[q]];
            }
            std::unique_ptr<DeviceBuf> fac;
            run_rsvd<R>(g, gp, in, p.eps, 24, 0, fac, st);
            pass_scratch.push_back(std::move(fac));
            pass_members.push_back(members);
            for (size_t q = 0; q < members.size(); ++q) {
                const int64_t k = members[q];
                aca_rank[k] = in[q].k;
                aca_u[k] = in[q].uoff;
                aca_v[k] = in[q].voff;
            }
            n_rsvd += (int32_t)members.size();
            t_aca += now_s() - tc;
            tc = now_s();
            compress_emit(0);
        } else {
            // Pass 0.  The blocks with many points run the split ACA, whose
            // steps the host drives; they go to a worker thread and their own
            // stream, so that the other blocks (one ACA launch) are finished
            // and recompressed meanwhile, as pass 0, and the split blocks
            // become pass 1.
            // This pays off once the split blocks hold some 200,000 points
            // together (a 20k-point sphere has 370,000); with fewer, the
            // second recompression round costs more than the overlap saves.
            std::vector<int64_t> big, small;
            int64_t big_points = 0;
            for (int64_t k : members) {
                const bool b = lm[k] + ln[k] >= kAcaBigPoints;
                (b ? big : small).push_back(k);
                if (b) big_points += lm[k] + ln[k];
            }
            std::vector<int64_t> next;
            size_t ps0 = 0;
            if (!p.unbatched && big_points >= 200000 && !small.empty()) {
                int dev = 0;
                HM_HIP_CHECK(hipGetDevice(&dev));
                auto split = std::async(std::launch::async, [&, dev]() {
                    HM_HIP_CHECK(hipSetDevice(dev));
                    return launch(big, aca_side);
                });
                std::exception_ptr err;
                int64_t first_bytes = 0;
                try {
                    AcaLaunch first = launch(small, st);
                    first_bytes = first.scratch_bytes;
                    next = finish(first);
                    compress_emit(0);
                } catch (...) {
                    err = std::current_exception();
                }
                // the worker uses this scope's state: wait for it before
                // anything unwinds (get() rethrows its own error)
                AcaLaunch second = split.get();
                if (err) std::rethrow_exception(err);
                if (!last) S.aca_scratch_bytes += first_bytes + second.scratch_bytes;
                const std::vector<int64_t> n2 = finish(second);
                next.insert(next.end(), n2.begin(), n2.end());
                ps0 = 1;
            } else {
                AcaLaunch first = launch(members, st);
                if (!last) S.aca_scratch_bytes += first.scratch_bytes;
                next = finish(first);
            }
            if (defer) {
                deferred.insert(deferred.end(), next.begin(), next.end());
                next.clear();
            }
            t_aca += now_s() - tc;
            tc = now_s();
            for (size_t ps = ps0;; ++ps) {
                const bool more = !next.empty();
                AcaLaunch rerun;
                if (more) rerun = launch(next, aca_side);   // runs beside ...
                compress_emit(ps);                          // ... this recompression
                if (!more) break;
                next = finish(rerun);
            }
        }
        ++n_chunks_done;
        // holding buffers whose blocks have all continued (their copies are done)
        holding.erase(std::remove_if(holding.begin(), holding.end(),
                                     [&](const Held &h) {
                                         for (const auto &bg : h.blocks)
                                             if (used_gen[bg.first] < bg.second) return false;
                                         return true;
                                     }),
                      holding.end());
        t_rc += now_s() - tc;
    }
    S.aca_chunks = n_chunks_done;
    S.n_overflow = overflow;
    S.n_capped = capped;
    S.n_rsvd = n_rsvd;
    if (capped)
        std::fprintf(stderr, "hmat: %d admissible blocks reached the ACA rank cap %d\n", capped,
                     budget_cap);
    S.n_fallback = fallbacks;
    S.n_model_hits = hits;
    S.t_aca = t_aca;
    S.t_recompress = t_rc;
    t = now_s();
    // ---- matvec plan -----------------------------------------------------------
    int32_t maxr_aca = 0, maxr = 0;
    int64_t sr_aca = 0, sr = 0;
    for (int64_t k = 0; k < nlr; ++k) {
        const int64_t b = lr_ids[k];
        const Block &B = M->blocks[b];
        LowRankBlk L;
        L.uoff = fu[k];
        L.voff = fv[k];
        L.toff = t_len;
        L.rb = tx.begin[B.row];
        L.m = lm[k];
        L.cb = ty.begin[B.col];
        L.n = ln[k];
        L.r = final_rank[k];
        L.ldu = padded_rows(rowpad, L.rb, L.m);
        L.ldv = even_up(L.r);
        L.pad = 0;
        t_len += L.r;
        M->block_slot[b] = (int32_t)M->h_lblk.size();
        M->off_a[b] = L.uoff;
        M->off_v[b] = L.voff;
        M->h_lblk.push_back(L);
        M->rank[b] = final_rank[k];
        M->rank_aca[b] = aca_rank[k];
        maxr_aca = std::max(maxr_aca, aca_rank[k]);
        maxr = std::max(maxr, final_rank[k]);
        sr_aca += aca_rank[k];
        sr += final_rank[k];
    }
    M->n_lblk = (int32_t)M->h_lblk.size();
    M->t_len = t_len;
    // tasks per leaf row cluster
    std::vector<int32_t> leaf_index(tx.nodes(), -1);
    std::vector<LeafRow> leaves;
    for (int32_t v = 0; v < tx.nodes(); ++v)
        if (tx.is_leaf(v)) {
            leaf_index[v] = (int32_t)leaves.size();
            leaves.push_back({tx.begin[v], tx.size(v), 0, 0});
            M->max_leaf = std::max(M->max_leaf, tx.size(v));
        }
    std::vector<std::vector<Task>> per_leaf(leaves.size());
    std::vector<int32_t> lv;
    for (int64_t b = 0; b < nb; ++b) {
        const Block &B = M->blocks[b];
        lv.clear();
        leaves_under(tx, B.row, lv);
        for (int32_t L : lv) {
            Task tk;
            tk.kind = B.kind == BLOCK_DENSE ? 0 : 1;
            tk.idx = M->block_slot[b];
            // padded row offset of leaf L inside the block's rows (even)
            tk.rowoff = padded_row(rowpad, tx.begin[B.row], tx.begin[L] - tx.begin[B.row], 0);
            tk.pad = 0;
            per_leaf[leaf_index[L]].push_back(tk);
        }
    }
    // Leaves in decreasing order of the bytes their workgroup streams, so that
    // the dispatcher hands out the longest accumulations first.
    std::vector<int64_t> leaf_bytes(leaves.size(), 0);
    for (size_t l = 0; l < leaves.size(); ++l)
        for (const Task &tk : per_leaf[l])
            leaf_bytes[l] += 3 * (int64_t)leaves[l].m *
                             (tk.kind == 0 ? 3 * (int64_t)M->h_dblk[tk.idx].n
                                           : (int64_t)M->h_lblk[tk.idx].r);
    std::vector<int32_t> leaf_order(leaves.size());
    std::iota(leaf_order.begin(), leaf_order.end(), 0);
    std::stable_sort(leaf_order.begin(), leaf_order.end(),
                     [&](int32_t a, int32_t b) { return leaf_bytes[a] > leaf_bytes[b]; });
    std::vector<LeafRow> sorted_leaves;
    std::vector<Task> tasks;
    for (int32_t l : leaf_order) {
        LeafRow L = leaves[l];
        L.tbeg = (int32_t)tasks.size();
        tasks.insert(tasks.end(), per_leaf[l].begin(), per_leaf[l].end());
        L.tend = (int32_t)tasks.size();
        sorted_leaves.push_back(L);
    }
    leaves.swap(sorted_leaves);
    M->n_leaves = (int32_t)leaves.size();
    build_project_plan(M, kProjRows, st);
    upload(M->d_lblk, M->h_lblk, st);
    upload(M->d_tasks, tasks, st);
    upload(M->d_leaves, leaves, st);
    if (M->p.prec == HM_C64) {
        // multi-RHS plan: accumulation waves ordered by the contraction length
        // of their leaf (longest first), projection items by chunk length
        std::vector<int64_t> leaf_cost(leaves.size(), 0);
        for (size_t l = 0; l < leaves.size(); ++l)
            for (int32_t q = leaves[l].tbeg; q < leaves[l].tend; ++q)
                leaf_cost[l] += tasks[q].kind == 0 ? 3 * (int64_t)M->h_dblk[tasks[q].idx].n
                                                   : (int64_t)M->h_lblk[tasks[q].idx].r;
        std::vector<MrAccItem> mracc;
        for (size_t l = 0; l < leaves.size(); ++l)
            for (int32_t r0 = 0; r0 < 3 * leaves[l].m; r0 += 16)
                mracc.push_back({(int32_t)l, r0, 0, 0});
        std::stable_sort(mracc.begin(), mracc.end(), [&](const MrAccItem &a, const MrAccItem &b) {
            return leaf_cost[a.leaf] > leaf_cost[b.leaf];
        });
        std::vector<MrProjItem> mrproj;
        std::vector<MrProjReduce> mrred;
        int32_t mslots = 0;
        for (int32_t i = 0; i < M->n_lblk; ++i) {
            const int32_t rows = 3 * M->h_lblk[i].n;
            const int32_t nch = (int32_t)ceil_div(rows, kMrChunk);
            for (int32_t j0 = 0; j0 < M->h_lblk[i].r; j0 += 16) {
                if (nch == 1) {
                    mrproj.push_back({i, j0, 0, rows, -1, 0});
                    continue;
                }
                mrred.push_back({i, j0, mslots, nch});
                for (int32_t ch = 0; ch < nch; ++ch)
                    mrproj.push_back({i, j0, ch * kMrChunk,
                                      std::min(kMrChunk, rows - ch * kMrChunk), mslots++, 0});
            }
        }
        std::stable_sort(mrproj.begin(), mrproj.end(),
                         [](const MrProjItem &a, const MrProjItem &b) { return a.klen > b.klen; });
        M->n_mracc = (int32_t)mracc.size();
        M->n_mrproj = (int32_t)mrproj.size();
        M->n_mrred = (int32_t)mrred.size();
        M->mr_nslots = mslots;
        upload(M->d_mracc, mracc, st);
        upload(M->d_mrproj, mrproj, st);
        upload(M->d_mrred, mrred, st);
    }
    M->ws_xc.alloc(3 * std::max(nx, ny) * sizeof(cplx<double>));
    M->ws_t.alloc(std::max<int64_t>(t_len, 1) * sizeof(cplx<double>));
    HM_HIP_CHECK(hipStreamSynchronize(st));
    S.t_plan = now_s() - t;
    S.lowrank_entries = lr_entries;
    S.max_rank_aca = maxr_aca;
    S.max_rank = maxr;
    S.sum_rank_aca = sr_aca;
    S.sum_rank = sr;
    S.storage_bytes = (dense_entries + lr_entries) * (int64_t)sizeof(cplx<R>);
    // algorithmic bytes: 9mn per dense tile + 3r(m+n) per low-rank block
    // (padding excluded) + one read of x + one write of y
    int64_t alg = 0;
    for (const auto &d : M->h_dblk) alg += 9 * (int64_t)d.m * d.n;
    for (const auto &L : M->h_lblk) alg += 3 * (int64_t)L.r * (L.m + L.n);
    S.matvec_bytes = (alg + 3 * nx + 3 * ny) * (int64_t)sizeof(cplx<R>);
    S.acc_waves = M->acc_waves;
    S.proj_rows = M->proj_rows;
}

}  // namespace

// The launches of y = A x on stream st (no allocation once the workspaces
// exist, no memset: safe to capture).
static void matvec_launches(const hm_matrix *A, const void *x, void *y, int32_t nrhs,
                            hipStream_t st) {
    if (A->p.prec == HM_C64 && nrhs >= kMrMinCols) {
        for (int32_t c0 = 0; c0 < nrhs; c0 += kMrPanel)
            launch_matvec_mrhs(A, x, nrhs, c0, std::min(kMrPanel, nrhs - c0), y, nrhs, st, nullptr);
        return;
    }
    for (int32_t c = 0; c < nrhs; ++c) {
        if (A->p.prec == HM_C64)
            launch_matvec_col<float, float>(A, x, nrhs, c, y, nrhs, nullptr, st);
        else
            launch_matvec_col<double, double>(A, x, nrhs, c, y, nrhs, nullptr, st);
    }
}

// Replays the captured launches of matvec_launches for (x, y, nrhs); a new
// key re-captures them on the matrix's private stream.
static void matvec_graph(const hm_matrix *A, const void *x, void *y, int32_t nrhs, hipStream_t st) {
    if (!A->g_exec || A->g_x != x || A->g_y != y || A->g_nrhs != nrhs) {
        if (A->g_exec) {
            HM_HIP_CHECK(hipGraphExecDestroy(A->g_exec));
            A->g_exec = nullptr;
        }
        if (!A->g_stream) HM_HIP_CHECK(hipStreamCreateWithFlags(&A->g_stream, hipStreamNonBlocking));
        if (A->p.prec == HM_C64 && nrhs >= kMrMinCols) ensure_mrhs_workspace(A);
        hipGraph_t graph = nullptr;
        HM_HIP_CHECK(hipStreamBeginCapture(A->g_stream, hipStreamCaptureModeThreadLocal));
        try {
            matvec_launches(A, x, y, nrhs, A->g_stream);
        } catch (...) {
            (void)hipStreamEndCapture(A->g_stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        HM_HIP_CHECK(hipStreamEndCapture(A->g_stream, &graph));
        const hipError_t e = hipGraphInstantiate(&A->g_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HM_HIP_CHECK(e);
        A->g_x = x;
        A->g_y = y;
        A->g_nrhs = nrhs;
    }
    HM_HIP_CHECK(hipGraphLaunch(A->g_exec, st));
}

extern "C" hm_status hm_matvec(const hm_matrix *A, const void *x, void *y, int32_t nrhs,
                               void *stream) {
    HM_API_BEGIN
    require(A != nullptr && x != nullptr && y != nullptr, "NULL argument");
    require(nrhs >= 1, "nrhs must be >= 1");
    if (A->plan_only) throw StatusError(HM_ERR_STATE, "matrix was built with plan_only");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (A->p.matvec_graph) {
        matvec_graph(A, x, y, nrhs, st);
        return HM_OK;
    }
    matvec_launches(A, x, y, nrhs, st);
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_residual(const hm_matrix *A, const void *b, const void *x, void *r,
                                 int32_t nrhs, void *stream) {
    HM_API_BEGIN
    require(A != nullptr && b != nullptr && x != nullptr && r != nullptr, "NULL argument");
    require(nrhs >= 1, "nrhs must be >= 1");
    if (A->plan_only) throw StatusError(HM_ERR_STATE, "matrix was built with plan_only");
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int32_t c = 0; c < nrhs; ++c) {
        if (A->p.prec == HM_C64)
            launch_matvec_col<float, double>(A, x, nrhs, c, r, nrhs,
                                             static_cast<const double *>(b), st);
        else
            launch_matvec_col<double, double>(A, x, nrhs, c, r, nrhs,
                                              static_cast<const double *>(b), st);
    }
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_profile_matvec(const hm_matrix *A, const void *x, void *y, int32_t reps,
                                       void *stream, double *kernel_ms, int64_t *kernel_bytes) {
    HM_API_BEGIN
    require(A != nullptr && x != nullptr && y != nullptr && reps >= 1, "bad arguments");
    if (A->plan_only) throw StatusError(HM_ERR_STATE, "matrix was built with plan_only");
    hipStream_t st = static_cast<hipStream_t>(stream);
    double ms[3] = {0, 0, 0};
    for (int32_t k = 0; k < reps; ++k) {
        if (A->p.prec == HM_C64)
            profile_matvec_col<float>(A, x, y, st, ms);
        else
            profile_matvec_col<double>(A, x, y, st, ms);
    }
    const int64_t es = (int64_t)elem_bytes(A->p.prec);
    int64_t vbytes = 0, ubytes = 0;
    for (const auto &L : A->h_lblk) {
        vbytes += 3 * (int64_t)L.n * L.r * es;
        ubytes += 3 * (int64_t)L.m * L.r * es;
    }
    int64_t dbytes = 0;
    for (const auto &d : A->h_dblk) dbytes += 9 * (int64_t)d.m * d.n * es;
    if (kernel_ms)
        for (int k = 0; k < 3; ++k) kernel_ms[k] = ms[k] / reps;
    if (kernel_bytes) {
        kernel_bytes[0] = 3 * A->ny * es;               // x read
        kernel_bytes[1] = vbytes;                       // V factors
        kernel_bytes[2] = dbytes + ubytes + 3 * A->nx * es;  // tiles + U factors + y write
    }
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_profile_matvec_multi(const hm_matrix *A, const void *x, void *y,
                                             int32_t reps, void *stream, double *kernel_ms,
                                             double *kernel_flops) {
    HM_API_BEGIN
    require(A != nullptr && x != nullptr && y != nullptr && reps >= 1, "bad arguments");
    if (A->plan_only) throw StatusError(HM_ERR_STATE, "matrix was built with plan_only");
    if (A->p.prec != HM_C64)
        throw StatusError(HM_ERR_STATE, "the multi-RHS panels need a complex64 operator");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t ev[4];
    for (auto &e : ev) HM_HIP_CHECK(hipEventCreate(&e));
    double ms[3] = {0, 0, 0};
    try {
        for (int32_t k = 0; k < reps; ++k) {
            launch_matvec_mrhs(A, x, kMrPanel, 0, kMrPanel, y, kMrPanel, st, ev);
            HM_HIP_CHECK(hipEventSynchronize(ev[3]));
            for (int q = 0; q < 3; ++q) {
                float t = 0;
                HM_HIP_CHECK(hipEventElapsedTime(&t, ev[q], ev[q + 1]));
                ms[q] += t;
            }
        }
    } catch (...) {
        for (auto &e : ev) (void)hipEventDestroy(e);
        throw;
    }
    for (auto &e : ev) HM_HIP_CHECK(hipEventDestroy(e));
    // algorithmic flops: 8 per complex multiply-add, 64 right-hand sides
    double vfl = 0, afl = 0;
    for (const auto &L : A->h_lblk) {
        vfl += 3.0 * L.n * L.r;
        afl += 3.0 * L.m * L.r;
    }
    for (const auto &d : A->h_dblk) afl += 9.0 * d.m * d.n;
    if (kernel_ms)
        for (int k = 0; k < 3; ++k) kernel_ms[k] = ms[k] / reps;
    if (kernel_flops) {
        kernel_flops[0] = 0;
        kernel_flops[1] = 8.0 * kMrPanel * vfl;
        kernel_flops[2] = 8.0 * kMrPanel * afl;
    }
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_autotune(hm_matrix *A, int32_t reps, void *stream, double *ms_table) {
    HM_API_BEGIN
    require(A != nullptr && reps >= 1, "bad arguments");
    if (A->plan_only) throw StatusError(HM_ERR_STATE, "matrix was built with plan_only");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t es = elem_bytes(A->p.prec);
    DeviceBuf xb, yb;
    xb.alloc(3 * std::max<int64_t>(A->ny, 1) * es);
    yb.alloc(3 * std::max<int64_t>(A->nx, 1) * es);
    HM_HIP_CHECK(hipMemsetAsync(xb.p, 0, 3 * std::max<int64_t>(A->ny, 1) * es, st));
    const int32_t waves[3] = {4, 8, 16}, chunks[3] = {256, 512, 1024};
    hipEvent_t e0, e1;
    HM_HIP_CHECK(hipEventCreate(&e0));
    HM_HIP_CHECK(hipEventCreate(&e1));
    double best = 1e300;
    int bw = 1, bc = 1;
    double table[9];
    try {
        for (int c = 0; c < 3; ++c) {
            build_project_plan(A, chunks[c], st);
            for (int w = 0; w < 3; ++w) {
                A->acc_waves = waves[w];
                for (int k = 0; k < 2; ++k) matvec_launches(A, xb.p, yb.p, 1, st);
                HM_HIP_CHECK(hipEventRecord(e0, st));
                for (int k = 0; k < reps; ++k) matvec_launches(A, xb.p, yb.p, 1, st);
                HM_HIP_CHECK(hipEventRecord(e1, st));
                HM_HIP_CHECK(hipEventSynchronize(e1));
                float ms = 0;
                HM_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
                table[3 * c + w] = ms / reps;
                if (table[3 * c + w] < best) {
                    best = table[3 * c + w];
                    bw = w;
                    bc = c;
                }
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    HM_HIP_CHECK(hipEventDestroy(e0));
    HM_HIP_CHECK(hipEventDestroy(e1));
    build_project_plan(A, chunks[bc], st);
    A->acc_waves = waves[bw];
    HM_HIP_CHECK(hipStreamSynchronize(st));
    if (A->g_exec) {   // a captured graph holds the old launch shape
        HM_HIP_CHECK(hipGraphExecDestroy(A->g_exec));
        A->g_exec = nullptr;
    }
    A->stats.acc_waves = A->acc_waves;
    A->stats.proj_rows = A->proj_rows;
    if (ms_table) std::memcpy(ms_table, table, sizeof(table));
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_info(const hm_matrix *A, hm_stats *s) {
    if (!A || !s) return HM_ERR_ARG;
    *s = A->stats;
    return HM_OK;
}

extern "C" hm_status hm_export_tree(const hm_matrix *A, int32_t which, int32_t *perm,
                                    int32_t *nodes, double *boxes) {
    HM_API_BEGIN
    require(A != nullptr, "NULL matrix");
    require(which == 0 || which == 1, "which must be 0 or 1");
    const ClusterTree &t = which == 0 ? A->rowtree() : A->coltree();
    if (perm) std::memcpy(perm, t.perm.data(), t.perm.size() * sizeof(int32_t));
    for (int32_t v = 0; v < t.nodes(); ++v) {
        if (nodes) {
            nodes[5 * v + 0] = t.begin[v];
            nodes[5 * v + 1] = t.end[v];
            nodes[5 * v + 2] = t.left[v];
            nodes[5 * v + 3] = t.right[v];
            nodes[5 * v + 4] = t.depth[v];
        }
        if (boxes)
            for (int a = 0; a < 3; ++a) {
                boxes[6 * v + a] = t.lo[3 * v + a];
                boxes[6 * v + 3 + a] = t.hi[3 * v + a];
            }
    }
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_export_blocklist(const hm_matrix *A, int32_t *blocks, int32_t *rank,
                                         int32_t *rank_aca) {
    HM_API_BEGIN
    require(A != nullptr, "NULL matrix");
    for (size_t b = 0; b < A->blocks.size(); ++b) {
        if (blocks) {
            blocks[3 * b] = A->blocks[b].row;
            blocks[3 * b + 1] = A->blocks[b].col;
            blocks[3 * b + 2] = A->blocks[b].kind;
        }
        if (rank) rank[b] = A->rank[b];
        if (rank_aca) rank_aca[b] = A->rank_aca[b];
    }
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_export_block(const hm_matrix *A, int64_t b, void *host_buf) {
    HM_API_BEGIN
    require(A != nullptr && host_buf != nullptr, "NULL argument");
    require(b >= 0 && b < (int64_t)A->blocks.size(), "block index out of range");
    if (A->plan_only) throw StatusError(HM_ERR_STATE, "matrix was built with plan_only");
    const size_t es = elem_bytes(A->p.prec);
    const Block &B = A->blocks[b];
    const int64_t m = A->rowtree().size(B.row), n = A->coltree().size(B.col);
    const int32_t rb = A->rowtree().begin[B.row];
    const int32_t *rowpad = A->rowpad.data();
    char *h = static_cast<char *>(host_buf);
    auto pr = [&](int64_t row) { return padded_row(rowpad, rb, (int32_t)(row / 3), (int)(row % 3)); };
    if (B.kind == BLOCK_DENSE) {
        const int64_t ld = padded_rows(rowpad, rb, (int32_t)m);
        std::vector<char> tmp(ld * 3 * n * es);
        HM_HIP_CHECK(hipMemcpy(tmp.data(), static_cast<char *>(A->dense.p) + A->off_a[b] * es,
                               tmp.size(), hipMemcpyDeviceToHost));
        for (int64_t c = 0; c < 3 * n; ++c)
            for (int64_t row = 0; row < 3 * m; ++row)
                std::memcpy(h + (c * 3 * m + row) * es, tmp.data() + (c * ld + pr(row)) * es, es);
    } else {
        const int64_t r = A->rank[b];
        if (r > 0) {
            const int64_t ldu = padded_rows(rowpad, rb, (int32_t)m), ldv = even_up((int32_t)r);
            std::vector<char> tu(ldu * r * es), tv(3 * n * ldv * es);
            HM_HIP_CHECK(hipMemcpy(tu.data(), static_cast<char *>(A->lr_base) + A->off_a[b] * es,
                                   tu.size(), hipMemcpyDeviceToHost));
            HM_HIP_CHECK(hipMemcpy(tv.data(), static_cast<char *>(A->lr_base) + A->off_v[b] * es,
                                   tv.size(), hipMemcpyDeviceToHost));
            for (int64_t c = 0; c < r; ++c)
                for (int64_t row = 0; row < 3 * m; ++row)
                    std::memcpy(h + (c * 3 * m + row) * es, tu.data() + (c * ldu + pr(row)) * es, es);
            // V is stored row-major; export it column-major.
            char *hv = h + 3 * m * r * es;
            for (int64_t row = 0; row < 3 * n; ++row)
                for (int64_t c = 0; c < r; ++c)
                    std::memcpy(hv + (c * 3 * n + row) * es, tv.data() + (row * ldv + c) * es, es);
        }
    }
    return HM_OK;
    HM_API_END
}

extern "C" void hm_destroy(hm_matrix *A) { delete A; }

extern "C" void hm_release_cache(void) { cache_release_all(); }
