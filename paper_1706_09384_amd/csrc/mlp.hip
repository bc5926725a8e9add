// Rank model: a 6 -> 64 -> 64 -> 1 ReLU network that predicts the ACA rank
// of an admissible block from its size and geometry, trained and evaluated
// with the library's own FP32 kernels.  A prediction only sizes the first
// ACA column budget and orders the ACA work; the ACA stopping test
// (eq. stop_part) still decides every rank.
//
// Parameters are packed W1 (64 x 6, row-major), b1, W2 (64 x 64), b2,
// W3 (1 x 64), b3.  Loss: mean squared error on the target log2(1 + r/3).
//
// Training step (one workgroup of 256 threads, one sample per thread, batch
// <= 256): the forward pass keeps z2 in registers and stages h1 and the
// output-layer gradient g2 = dL/dz2 in LDS (row stride 65 floats: no bank
// conflicts); the weight gradients are then batch sums read from LDS, each
// thread owning 16 entries of dW2 plus a few others, and the same thread
// applies the Adam update to the entries it owns.  Larger sample sets for the
// gradient check are split over workgroups whose partial sums are added in
// a fixed order.
#include <algorithm>
#include <cmath>
#include <random>
#include <vector>

#include "internal.hpp"

namespace hm {

namespace {

constexpr int kIn = 6, kHid = 64, kThreads = 256, kPad = 65;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kHid, kParams = oB3 + 1;
static_assert(kParams == HM_RANK_MODEL_PARAMS, "parameter packing");

__global__ void __launch_bounds__(256) mlp_predict_kernel(const float *__restrict__ w,
                                                          const float *__restrict__ X,
                                                          float *__restrict__ out, int64_t n) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float x[kIn];
#pragma unroll
    for (int j = 0; j < kIn; ++j) x[j] = X[s * kIn + j];
    float h1[kHid];
#pragma unroll
    for (int o = 0; o < kHid; ++o) {
        float z = w[oB1 + o];
#pragma unroll
        for (int j = 0; j < kIn; ++j) z += w[oW1 + o * kIn + j] * x[j];
        h1[o] = fmaxf(z, 0.f);
    }
    float y = w[oB3];
    for (int o = 0; o < kHid; ++o) {
        float z = w[oB2 + o];
#pragma unroll
        for (int i = 0; i < kHid; ++i) z += w[oW2 + o * kHid + i] * h1[i];
        y += w[oW3 + o] * fmaxf(z, 0.f);
    }
    out[s] = y;
}

struct GradLds {
    float H[kThreads * kPad];    // h1, later g1 = dL/dz1
    float G[kThreads * kPad];    // g2 = dL/dz2, later h2
    float X[kThreads * kIn];
    float gout[kThreads];        // dL/d out
    float red[kThreads];
};

// Gradient of sum_s (out_s - t_s)^2 * scale over the samples of this
// workgroup (sample ids from idx, or s0 + local id when idx is null).
// MODE 0: write the partial gradient and loss; MODE 1: Adam update in place.
template <int MODE>
__global__ void __launch_bounds__(kThreads) mlp_grad_kernel(
    float *__restrict__ w, const float *__restrict__ Xg, const float *__restrict__ tg,
    const int32_t *__restrict__ idx, int64_t s0, int64_t nsamp, float scale,
    float *__restrict__ gpart, float *__restrict__ lpart,
    // Adam state (MODE 1)
    float *__restrict__ am, float *__restrict__ av, float lr, float b1c, float b2c) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    GradLds &L = *reinterpret_cast<GradLds *>(smem_raw);
    const int tid = threadIdx.x;
    const int64_t base = s0 + (int64_t)blockIdx.x * kThreads;
    const bool valid = base + tid < nsamp;
    int64_t sid = 0;
    if (valid) sid = idx ? idx[base + tid] : base + tid;
    // ---- forward (thread = sample) ----
    float x[kIn];
#pragma unroll
    for (int j = 0; j < kIn; ++j) x[j] = valid ? Xg[sid * kIn + j] : 0.f;
#pragma unroll
    for (int j = 0; j < kIn; ++j) L.X[tid * kIn + j] = x[j];
    float h1[kHid];
#pragma unroll
    for (int o = 0; o < kHid; ++o) {
        float z = w[oB1 + o];
#pragma unroll
        for (int j = 0; j < kIn; ++j) z += w[oW1 + o * kIn + j] * x[j];
        h1[o] = fmaxf(z, 0.f);
        L.H[tid * kPad + o] = h1[o];
    }
    float z2[kHid];
    float y = w[oB3];
#pragma unroll
    for (int o = 0; o < kHid; ++o) {
        float z = w[oB2 + o];
#pragma unroll
        for (int i = 0; i < kHid; ++i) z += w[oW2 + o * kHid + i] * h1[i];
        z2[o] = z;
        y += w[oW3 + o] * fmaxf(z, 0.f);
    }
    const float diff = valid ? y - tg[sid] : 0.f;
    const float go = 2.f * scale * diff;
    L.gout[tid] = go;
    L.red[tid] = diff * diff;
#pragma unroll
    for (int o = 0; o < kHid; ++o) L.G[tid * kPad + o] = z2[o] > 0.f ? go * w[oW3 + o] : 0.f;
    __syncthreads();
    // ---- dW2 = G^T H, db2 = sum G (entries e = tid + 256 q) ----
    float gw2[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + kThreads * q, o = e / kHid, i = e % kHid;
        float acc = 0.f;
        for (int s = 0; s < kThreads; ++s) acc += L.G[s * kPad + o] * L.H[s * kPad + i];
        gw2[q] = acc;
    }
    float gb2 = 0.f;
    if (tid < kHid)
        for (int s = 0; s < kThreads; ++s) gb2 += L.G[s * kPad + tid];
    // ---- g1 = (W2^T g2) * (h1 > 0), own sample ----
    float g1[kHid];
#pragma unroll
    for (int i = 0; i < kHid; ++i) g1[i] = 0.f;
    for (int o = 0; o < kHid; ++o) {
        const float g = L.G[tid * kPad + o];
#pragma unroll
        for (int i = 0; i < kHid; ++i) g1[i] += g * w[oW2 + o * kHid + i];
    }
    __syncthreads();   // every read of H and G above is done
#pragma unroll
    for (int i = 0; i < kHid; ++i) {
        const float hv = L.H[tid * kPad + i];   // own row: h1 of this sample
        L.H[tid * kPad + i] = hv > 0.f ? g1[i] : 0.f;
    }
#pragma unroll
    for (int o = 0; o < kHid; ++o) L.G[tid * kPad + o] = fmaxf(z2[o], 0.f);
    __syncthreads();
    // ---- dW1 = g1^T X, db1 = sum g1, dW3 = gout^T h2, db3 = sum gout ----
    float gw1[2] = {0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = tid + kThreads * q;
        if (e < kHid * kIn) {
            const int o = e / kIn, j = e % kIn;
            float acc = 0.f;
            for (int s = 0; s < kThreads; ++s) acc += L.H[s * kPad + o] * L.X[s * kIn + j];
            gw1[q] = acc;
        }
    }
    float gb1 = 0.f, gw3 = 0.f, gb3 = 0.f;
    if (tid < kHid) {
        for (int s = 0; s < kThreads; ++s) {
            gb1 += L.H[s * kPad + tid];
            gw3 += L.gout[s] * L.G[s * kPad + tid];
        }
    } else if (tid == kHid) {
        for (int s = 0; s < kThreads; ++s) gb3 += L.gout[s];
    }
    // loss partial (fixed tree order)
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        __syncthreads();
        if (tid < h) L.red[tid] += L.red[tid + h];
    }
    __syncthreads();
    // ---- output: partial sums, or Adam on the entries this thread owns ----
    auto emit = [&](int p, float g) {
        if (MODE == 0) {
            gpart[(int64_t)blockIdx.x * kParams + p] = g;
        } else {
            const float m = 0.9f * am[p] + 0.1f * g;
            const float v = 0.999f * av[p] + 0.001f * g * g;
            am[p] = m;
            av[p] = v;
            w[p] -= lr * (m / b1c) / (sqrtf(v / b2c) + 1e-8f);
        }
    };
    // Each parameter is read above by every thread before any thread writes
    // it here; the barrier before this point orders those reads and writes.
#pragma unroll
    for (int q = 0; q < 16; ++q) emit(oW2 + tid + kThreads * q, gw2[q]);
#pragma unroll
    for (int q = 0; q < 2; ++q)
        if (tid + kThreads * q < kHid * kIn) emit(oW1 + tid + kThreads * q, gw1[q]);
    if (tid < kHid) {
        emit(oB2 + tid, gb2);
        emit(oB1 + tid, gb1);
        emit(oW3 + tid, gw3);
    } else if (tid == kHid) {
        emit(oB3, gb3);
    }
    if (MODE == 0 && tid == 0) lpart[blockIdx.x] = L.red[0] * scale;
    if (MODE == 1 && tid == 0 && lpart) lpart[0] = L.red[0] * scale;
}

// Sum of the per-workgroup partial gradients, in workgroup order.
__global__ void mlp_reduce_kernel(const float *__restrict__ gpart, const float *__restrict__ lpart,
                                  int32_t nblk, float *__restrict__ g, float *__restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kParams) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += gpart[(int64_t)b * kParams + p];
        g[p] = s;
    }
    if (p == 0) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += lpart[b];
        *loss = s;
    }
}

void set_grad_lds() {
    static bool done = false;
    if (done) return;
    HM_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(&mlp_grad_kernel<0>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)sizeof(GradLds)));
    HM_HIP_CHECK(hipFuncSetAttribute(reinterpret_cast<const void *>(&mlp_grad_kernel<1>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)sizeof(GradLds)));
    done = true;
}

template <typename T>
void to_device(DeviceBuf &d, const T *h, size_t n, hipStream_t st) {
    d.alloc(std::max<size_t>(n, 1) * sizeof(T));
    if (n) HM_HIP_CHECK(hipMemcpyAsync(d.p, h, n * sizeof(T), hipMemcpyHostToDevice, st));
    HM_HIP_CHECK(hipStreamSynchronize(st));   // h may be pageable and short-lived
}

}  // namespace

// Features of every admissible block, in the order of the block list.
void rank_features(const hm_matrix *M, std::vector<float> &feats, std::vector<int64_t> &ids) {
    const ClusterTree &tx = M->rowtree(), &ty = M->coltree();
    const double k = M->p.omega * std::sqrt(M->p.rho / M->p.mu);   // kappa_s
    const double le = std::log10(M->p.eps);
    feats.clear();
    ids.clear();
    for (int64_t b = 0; b < (int64_t)M->blocks.size(); ++b) {
        const Block &B = M->blocks[b];
        if (B.kind != BLOCK_LOWRANK) continue;
        ids.push_back(b);
        feats.push_back((float)std::log((double)tx.size(B.row)));
        feats.push_back((float)std::log((double)ty.size(B.col)));
        feats.push_back((float)(k * box_diam(tx, B.row)));
        feats.push_back((float)(k * box_diam(ty, B.col)));
        feats.push_back((float)(k * box_dist(tx, B.row, ty, B.col)));
        feats.push_back((float)le);
    }
}

void rank_predict(const float *w_host, const std::vector<float> &feats, std::vector<float> &pred,
                  hipStream_t st) {
    const int64_t n = (int64_t)feats.size() / kIn;
    pred.assign(n, 0.f);
    if (n == 0) return;
    DeviceBuf dw, dx, dy;
    to_device(dw, w_host, kParams, st);
    to_device(dx, feats.data(), feats.size(), st);
    dy.alloc(n * sizeof(float));
    hipLaunchKernelGGL(mlp_predict_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st,
                       dw.as<float>(), dx.as<float>(), dy.as<float>(), n);
    HM_HIP_CHECK(hipGetLastError());
    HM_HIP_CHECK(hipMemcpyAsync(pred.data(), dy.p, n * sizeof(float), hipMemcpyDeviceToHost, st));
    HM_HIP_CHECK(hipStreamSynchronize(st));
}

}  // namespace hm

using namespace hm;

extern "C" hm_status hm_rank_samples(const hm_matrix *A, float *feats, int32_t *ranks) {
    HM_API_BEGIN
    if (!A || !feats || !ranks) throw StatusError(HM_ERR_ARG, "NULL argument");
    std::vector<float> f;
    std::vector<int64_t> ids;
    rank_features(A, f, ids);
    std::copy(f.begin(), f.end(), feats);
    // a plan_only matrix has trees and blocks but no ACA: ranks are -1
    for (size_t q = 0; q < ids.size(); ++q) ranks[q] = A->plan_only ? -1 : A->rank_aca[ids[q]];
    set_error("");
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_rank_model_predict(const float *weights_host, const float *feats,
                                           float *pred, int64_t n, void *stream) {
    HM_API_BEGIN
    if (!weights_host || (n > 0 && (!feats || !pred)) || n < 0)
        throw StatusError(HM_ERR_ARG, "bad arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n == 0) return HM_OK;
    DeviceBuf dw;
    to_device(dw, weights_host, kParams, st);
    hipLaunchKernelGGL(mlp_predict_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st,
                       dw.as<float>(), feats, pred, n);
    HM_HIP_CHECK(hipGetLastError());
    HM_HIP_CHECK(hipStreamSynchronize(st));   // dw is freed on return
    set_error("");
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_rank_model_grad(const float *weights_host, const float *feats,
                                        const float *targets, int64_t n, float *loss,
                                        float *grad_host, void *stream) {
    HM_API_BEGIN
    if (!weights_host || !feats || !targets || !loss || !grad_host || n < 1)
        throw StatusError(HM_ERR_ARG, "bad arguments");
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_grad_lds();
    const int32_t nblk = (int32_t)ceil_div(n, kThreads);
    DeviceBuf dw, gpart, lpart, g, l;
    to_device(dw, weights_host, kParams, st);
    gpart.alloc((size_t)nblk * kParams * sizeof(float));
    lpart.alloc(nblk * sizeof(float));
    g.alloc(kParams * sizeof(float));
    l.alloc(sizeof(float));
    hipLaunchKernelGGL(mlp_grad_kernel<0>, dim3(nblk), dim3(kThreads), sizeof(GradLds), st,
                       dw.as<float>(), feats, targets, nullptr, (int64_t)0, n, 1.f / (float)n,
                       gpart.as<float>(), lpart.as<float>(), nullptr, nullptr, 0.f, 1.f, 1.f);
    HM_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((unsigned)ceil_div(kParams, 256)), dim3(256), 0, st,
                       gpart.as<float>(), lpart.as<float>(), nblk, g.as<float>(), l.as<float>());
    HM_HIP_CHECK(hipGetLastError());
    HM_HIP_CHECK(hipMemcpyAsync(grad_host, g.p, kParams * sizeof(float), hipMemcpyDeviceToHost, st));
    HM_HIP_CHECK(hipMemcpyAsync(loss, l.p, sizeof(float), hipMemcpyDeviceToHost, st));
    HM_HIP_CHECK(hipStreamSynchronize(st));
    set_error("");
    return HM_OK;
    HM_API_END
}

extern "C" hm_status hm_rank_model_train(const float *feats, const int32_t *ranks, int64_t n,
                                         float *weights, int32_t epochs, int32_t batch, float lr,
                                         uint64_t seed, float *loss_out, void *stream) {
    HM_API_BEGIN
    if (!feats || !ranks || !weights || n < 1 || epochs < 1 || batch < 1 || batch > kThreads ||
        !(lr > 0.f))
        throw StatusError(HM_ERR_ARG, "bad arguments (need n >= 1, epochs >= 1, 1 <= batch <= 256, lr > 0)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    set_grad_lds();
    std::vector<float> t(n);
    for (int64_t s = 0; s < n; ++s) t[s] = (float)std::log2(1.0 + ranks[s] / 3.0);
    // every epoch's sample order, from a seeded 64-bit Mersenne twister
    std::vector<int32_t> order((size_t)epochs * n);
    std::mt19937_64 rng(seed);
    std::vector<int32_t> p(n);
    for (int64_t s = 0; s < n; ++s) p[s] = (int32_t)s;
    for (int32_t e = 0; e < epochs; ++e) {
        for (int64_t s = n - 1; s > 0; --s) {
            const int64_t j = (int64_t)(rng() % (uint64_t)(s + 1));
            std::swap(p[s], p[j]);
        }
        std::copy(p.begin(), p.end(), order.begin() + (size_t)e * n);
    }
    const int64_t steps_per_epoch = ceil_div(n, batch);
    const int64_t nsteps = steps_per_epoch * epochs;
    DeviceBuf dw, dx, dt, dord, dm, dv, dl;
    to_device(dw, weights, kParams, st);
    to_device(dx, feats, (size_t)n * kIn, st);
    to_device(dt, t.data(), t.size(), st);
    to_device(dord, order.data(), order.size(), st);
    dm.alloc(kParams * sizeof(float));
    dv.alloc(kParams * sizeof(float));
    dl.alloc(nsteps * sizeof(float));
    HM_HIP_CHECK(hipMemsetAsync(dm.p, 0, kParams * sizeof(float), st));
    HM_HIP_CHECK(hipMemsetAsync(dv.p, 0, kParams * sizeof(float), st));
    int64_t step = 0;
    for (int32_t e = 0; e < epochs; ++e)
        for (int64_t q = 0; q < steps_per_epoch; ++q, ++step) {
            const int64_t b0 = q * batch, nb = std::min<int64_t>(batch, n - b0);
            const double k = (double)(step + 1);
            const float b1c = (float)(1.0 - std::pow(0.9, k));
            const float b2c = (float)(1.0 - std::pow(0.999, k));
            // one workgroup: samples order[e n + b0 .. + nb)
            hipLaunchKernelGGL(mlp_grad_kernel<1>, dim3(1), dim3(kThreads), sizeof(GradLds), st,
                               dw.as<float>(), dx.as<float>(), dt.as<float>(),
                               dord.as<int32_t>() + (size_t)e * n + b0, (int64_t)0, nb,
                               1.f / (float)nb, nullptr, dl.as<float>() + step, dm.as<float>(),
                               dv.as<float>(), lr, b1c, b2c);
            HM_HIP_CHECK(hipGetLastError());
        }
    std::vector<float> ls(nsteps);
    HM_HIP_CHECK(hipMemcpyAsync(ls.data(), dl.p, nsteps * sizeof(float), hipMemcpyDeviceToHost, st));
    HM_HIP_CHECK(hipMemcpyAsync(weights, dw.p, kParams * sizeof(float), hipMemcpyDeviceToHost, st));
    HM_HIP_CHECK(hipStreamSynchronize(st));
    if (loss_out)
        for (int32_t e = 0; e < epochs; ++e) {
            double s = 0;
            for (int64_t q = 0; q < steps_per_epoch; ++q) {
                const int64_t nb = std::min<int64_t>(batch, n - q * batch);
                s += (double)ls[e * steps_per_epoch + q] * nb;
            }
            loss_out[e] = (float)(s / n);
        }
    set_error("");
    return HM_OK;
    HM_API_END
}
