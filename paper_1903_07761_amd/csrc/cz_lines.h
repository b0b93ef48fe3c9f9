// One level of the W4 / W4_li / W3_ai wavelet transform along a single line
// held in registers (arXiv 1903.07761, Sec. 2.3 "Wavelet types").
//
// A line of n samples becomes [n/2 coarse | n/2 details].  Every stencil is
// expanded at compile time (fold expressions over the sample index), so a line
// stays in VGPRs and each weight is an immediate.  Weighted sums are formed
// left to right in ascending source index, every step rounded in T; the file
// is compiled with contraction off, so no multiply-add is fused.
//
//   W4     detail m = odd m - P_m(evens): the cubic through the four nearest
//          existing evens, evaluated at m + 1/2 (coarse coordinates).  Rows:
//            m = 0        (5, 15, -5, 1)/16      on e0..e3
//            interior     (-1, 9, 9, -1)/16      on e_m-1..e_m+2
//            m = h-2      (1, -5, 15, 5)/16      on e_h-4..e_h-1
//            m = h-1      (-5, 21, -35, 35)/16   on e_h-4..e_h-1
//          coarse k = even k.
//   W4_li  W4, then coarse k += (-1, 9, 9, -1)/32 over d_k-2..d_k+1, keeping
//          the details that exist (Sweldens' update, truncated at the ends).
//   W3_ai  coarse k = (v[2k] + v[2k+1]) / 2; detail k = v[2k] - the average
//          over the left half-cell of the quadratic matching three coarse
//          averages:  k = 0 (11, -4, 1)/8 on C0..C2; interior (1, 8, -1)/8 on
//          C_k-1..C_k+1; k = h-1 (-1, 4, 5)/8 on C_h-3..C_h-1.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace czk {

enum { W4 = 0, W4LI = 1, W3AI = 2 };

template <int... I>
using iseq = std::integer_sequence<int, I...>;
template <int N>
using make_iseq = std::make_integer_sequence<int, N>;

// W4 / W4_li predict of odd sample M from the evens e[0..H).
template <typename T, int H, int M>
__device__ __forceinline__ T w4_pred(const T *e)
{
    static_assert(H >= 4, "a level needs at least four coarse samples");
    if constexpr (M == 0)
        return ((T(0.3125) * e[0] + T(0.9375) * e[1]) + T(-0.3125) * e[2]) + T(0.0625) * e[3];
    else if constexpr (M == H - 1)
        return ((T(-0.3125) * e[H - 4] + T(1.3125) * e[H - 3]) + T(-2.1875) * e[H - 2]) + T(2.1875) * e[H - 1];
    else if constexpr (M == H - 2)
        return ((T(0.0625) * e[H - 4] + T(-0.3125) * e[H - 3]) + T(0.9375) * e[H - 2]) + T(0.3125) * e[H - 1];
    else
        return ((T(-0.0625) * e[M - 1] + T(0.5625) * e[M]) + T(0.5625) * e[M + 1]) + T(-0.0625) * e[M + 2];
}

// W4_li update of even K from the details d[0..H).
template <typename T, int H, int K>
__device__ __forceinline__ T w4li_update(const T *d)
{
    constexpr T a = T(-0.03125), b = T(0.28125);  // -1/32, 9/32
    if constexpr (K == 0)
        return b * d[0] + a * d[1];
    else if constexpr (K == 1)
        return (b * d[0] + b * d[1]) + a * d[2];
    else if constexpr (K == H - 1)
        return (a * d[H - 3] + b * d[H - 2]) + b * d[H - 1];
    else
        return ((a * d[K - 2] + b * d[K - 1]) + b * d[K]) + a * d[K + 1];
}

// W3_ai predict of the left child of coarse cell K from the averages C[0..H).
template <typename T, int H, int K>
__device__ __forceinline__ T w3_pred(const T *C)
{
    static_assert(H >= 3, "a level needs at least three coarse cells");
    if constexpr (K == 0)
        return (T(1.375) * C[0] + T(-0.5) * C[1]) + T(0.125) * C[2];
    else if constexpr (K == H - 1)
        return (T(-0.125) * C[H - 3] + T(0.5) * C[H - 2]) + T(0.625) * C[H - 1];
    else
        return (T(0.125) * C[K - 1] + C[K]) + T(-0.125) * C[K + 1];
}

template <typename T, int H, int... M>
__device__ __forceinline__ void w4_details(const T *e, const T *o, T *d, iseq<M...>)
{
    ((d[M] = o[M] - w4_pred<T, H, M>(e)), ...);
}

template <typename T, int H, int... K>
__device__ __forceinline__ void w4li_lift(T *s, const T *d, iseq<K...>)
{
    ((s[K] = s[K] + w4li_update<T, H, K>(d)), ...);
}

template <typename T, int H, int... K>
__device__ __forceinline__ void w4li_unlift(T *s, const T *d, iseq<K...>)
{
    ((s[K] = s[K] - w4li_update<T, H, K>(d)), ...);
}

template <typename T, int H, int... M>
__device__ __forceinline__ void w4_odds(const T *e, const T *d, T *v, iseq<M...>)
{
    ((v[2 * M + 1] = d[M] + w4_pred<T, H, M>(e)), ...);
}

template <typename T, int H, int... K>
__device__ __forceinline__ void w3_details(const T *v, const T *C, T *d, iseq<K...>)
{
    ((d[K] = v[2 * K] - w3_pred<T, H, K>(C)), ...);
}

template <typename T, int H, int K>
__device__ __forceinline__ void w3_pair(const T *C, const T *d, T *v)
{
    T a = w3_pred<T, H, K>(C) + d[K];
    v[2 * K] = a;
    v[2 * K + 1] = (C[K] + C[K]) - a;
}

template <typename T, int H, int... K>
__device__ __forceinline__ void w3_pairs(const T *C, const T *d, T *v, iseq<K...>)
{
    (w3_pair<T, H, K>(C, d, v), ...);
}

// Forward level: v[0..n) -> [coarse | details], in place.
template <typename T, int S, int n>
__device__ __forceinline__ void line_fwd(T *v)
{
    constexpr int H = n / 2;
    T a[H], d[H];
    if constexpr (S == W3AI) {
#pragma unroll
        for (int k = 0; k < H; ++k)
            a[k] = (v[2 * k] + v[2 * k + 1]) * T(0.5);
        w3_details<T, H>(v, a, d, make_iseq<H>{});
    } else {
        T o[H];
#pragma unroll
        for (int k = 0; k < H; ++k) {
            a[k] = v[2 * k];
            o[k] = v[2 * k + 1];
        }
        w4_details<T, H>(a, o, d, make_iseq<H>{});
        if constexpr (S == W4LI)
            w4li_lift<T, H>(a, d, make_iseq<H>{});
    }
#pragma unroll
    for (int k = 0; k < H; ++k) {
        v[k] = a[k];
        v[H + k] = d[k];
    }
}

// Inverse level: [coarse | details] -> v[0..n), in place.
template <typename T, int S, int n>
__device__ __forceinline__ void line_inv(T *v)
{
    constexpr int H = n / 2;
    T s[H], d[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
        s[k] = v[k];
        d[k] = v[H + k];
    }
    if constexpr (S == W3AI) {
        w3_pairs<T, H>(s, d, v, make_iseq<H>{});
    } else {
        if constexpr (S == W4LI)
            w4li_unlift<T, H>(s, d, make_iseq<H>{});
#pragma unroll
        for (int k = 0; k < H; ++k)
            v[2 * k] = s[k];
        w4_odds<T, H>(s, d, v, make_iseq<H>{});
    }
}

}  // namespace czk
