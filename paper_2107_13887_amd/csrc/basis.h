// Wendland compactly supported basis functions (Table 1), shared by the kernel sums, the greedy
// and the dense factorization. Each is written in t = max(1 - eta, 0), so it is exactly zero
// from eta = 1 on, and each takes the value 1 at eta = 0:
//   C0: t^2,  C2: t^4 (4 eta + 1) (eq. (2)),  C4: t^6 (35/3 eta^2 + 6 eta + 1),
//   C6: t^8 (32 eta^3 + 25 eta^2 + 8 eta + 1).
#pragma once

#include <hip/hip_runtime.h>

#include "rbfdef.h"

namespace rbf {

template <int BASIS, typename T>
__device__ __forceinline__ T wendland_t(T eta, T t)
{
    const T t2 = t * t;
    if constexpr (BASIS == RBF_WENDLAND_C0) {
        return t2;
    } else if constexpr (BASIS == RBF_WENDLAND_C2) {
        return (t2 * t2) * __builtin_fma(T(4), eta, T(1));
    } else if constexpr (BASIS == RBF_WENDLAND_C4) {
        const T t4 = t2 * t2;
        return (t4 * t2) * __builtin_fma(__builtin_fma(T(35.0 / 3.0), eta, T(6)), eta, T(1));
    } else {
        const T t4 = t2 * t2;
        return (t4 * t4) * __builtin_fma(__builtin_fma(__builtin_fma(T(32), eta, T(25)), eta, T(8)), eta, T(1));
    }
}

// The same functions written in t alone (eta = 1 - t), for a caller that forms t without eta:
// tc = max(t, 0) carries the compact support and t the polynomial factor (t may be tc itself:
// where they differ the product is zero either way):
//   C0: tc^2,  C2: tc^4 (5 - 4 t),  C4: tc^6 (35/3 t^2 - 88/3 t + 56/3),
//   C6: tc^8 (-32 t^3 + 121 t^2 - 154 t + 66).
template <int BASIS, typename T>
__device__ __forceinline__ T wendland_tform(T tc, T t)
{
    const T t2 = tc * tc;
    if constexpr (BASIS == RBF_WENDLAND_C0) {
        return t2;
    } else if constexpr (BASIS == RBF_WENDLAND_C2) {
        return (t2 * t2) * __builtin_fma(T(-4), t, T(5));
    } else if constexpr (BASIS == RBF_WENDLAND_C4) {
        const T t4 = t2 * t2;
        return (t4 * t2) * __builtin_fma(__builtin_fma(T(35.0 / 3.0), t, T(-88.0 / 3.0)), t, T(56.0 / 3.0));
    } else {
        const T t4 = t2 * t2;
        return (t4 * t4) *
               __builtin_fma(__builtin_fma(__builtin_fma(T(-32), t, T(121)), t, T(-154)), t, T(66));
    }
}

// Runtime selection (uniform across a launch), FP64.
__device__ __forceinline__ double wendland(int32_t basis, double eta)
{
    const double t = fmax(1.0 - eta, 0.0);
    switch (basis) {
    case RBF_WENDLAND_C0: return wendland_t<RBF_WENDLAND_C0>(eta, t);
    case RBF_WENDLAND_C4: return wendland_t<RBF_WENDLAND_C4>(eta, t);
    case RBF_WENDLAND_C6: return wendland_t<RBF_WENDLAND_C6>(eta, t);
    default: return wendland_t<RBF_WENDLAND_C2>(eta, t);
    }
}

inline bool basis_valid(int32_t b)
{
    return b == RBF_WENDLAND_C0 || b == RBF_WENDLAND_C2 || b == RBF_WENDLAND_C4 || b == RBF_WENDLAND_C6;
}

}  // namespace rbf
