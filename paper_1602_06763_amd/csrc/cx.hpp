// Complex scalars of the c/z instances (LAPACK storage: a (real, imaginary)
// pair per element) and the arithmetic every complex kernel shares, so that
// all of them round alike: products as written (re = ar·br − ai·bi,
// im = ar·bi + ai·br), quotients a·conj(p) / |p|², and |re| + |im| as the
// pivot magnitude (LAPACK's izamax rule).
#pragma once

#include <hip/hip_runtime.h>

namespace rl {

template <typename R>
struct alignas(2 * sizeof(R)) cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return cx<R>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> cconj(cx<R> a) {
    return cx<R>{a.re, -a.im};
}
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) {
    return cx<R>{a.re - b.re, a.im - b.im};
}
template <typename R>
__device__ __forceinline__ cx<R> cdiv(cx<R> a, cx<R> p) {
    const R den = p.re * p.re + p.im * p.im;
    const cx<R> q = cmul(a, cconj(p));
    return cx<R>{q.re / den, q.im / den};
}
template <typename R>
__device__ __forceinline__ R cabs1(cx<R> z) {
    return fabs(z.re) + fabs(z.im);
}

constexpr int kZLuLeaf = 16;   // complex LU panel width

}  // namespace rl
