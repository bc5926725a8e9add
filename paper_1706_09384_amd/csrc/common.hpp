// Shared definitions of the hmat library: complex arithmetic usable on host
// and device, error plumbing, and small helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/hmat.h"

namespace hm {

template <typename R>
struct cplx {
    R re, im;
};

template <typename R>
__host__ __device__ inline cplx<R> mk(R a, R b) { return cplx<R>{a, b}; }
template <typename R>
__host__ __device__ inline cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ inline cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ inline cplx<R> operator*(cplx<R> a, cplx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ inline cplx<R> operator*(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__host__ __device__ inline cplx<R> conj(cplx<R> a) { return {a.re, -a.im}; }
template <typename R>
__host__ __device__ inline R abs2(cplx<R> a) { return a.re * a.re + a.im * a.im; }
// a * conj(b)
template <typename R>
__host__ __device__ inline cplx<R> mulc(cplx<R> a, cplx<R> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// conj(a) * b
template <typename R>
__host__ __device__ inline cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// acc += a * b
template <typename R>
__host__ __device__ inline void fma_(cplx<R> &acc, cplx<R> a, cplx<R> b) {
    acc.re += a.re * b.re - a.im * b.im;
    acc.im += a.re * b.im + a.im * b.re;
}
// acc -= a * conj(b)
template <typename R>
__host__ __device__ inline void fms_conj(cplx<R> &acc, cplx<R> a, cplx<R> b) {
    acc.re -= a.re * b.re + a.im * b.im;
    acc.im -= a.im * b.re - a.re * b.im;
}
template <typename D, typename S>
__host__ __device__ inline cplx<D> cvt(cplx<S> a) { return {D(a.re), D(a.im)}; }

// Per-thread last-error message (set by the API layer).
void set_error(const std::string &msg);

}  // namespace hm

#define HM_HIP_CHECK(expr)                                                              \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess) {                                                         \
            throw hm::HipError(std::string(#expr) + ": " + hipGetErrorString(_e), _e); \
        }                                                                               \
    } while (0)

namespace hm {

struct HipError {
    std::string msg;
    hipError_t code;
    HipError(std::string m, hipError_t c) : msg(std::move(m)), code(c) {}
};

struct StatusError {
    hm_status status;
    std::string msg;
    StatusError(hm_status s, std::string m) : status(s), msg(std::move(m)) {}
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace hm
