// routines.hip -- the SU(3) routines of Table 1 as GPU kernels, one thread per
// call over n independent calls (a microbenchmark of each routine on its own,
// as the paper times them one by one, and a check of each against the oracle).
//
// Operands are structure-of-arrays planes of complex numbers: a vector is
// [3][n], a matrix [9][n] (element 3 i + j), a four-direction operand [4][..][n].
// The Wilson half-vector routines of Table 1 are not built (staggered only).
#include "../../include/lgt.h"
#include "fields.hpp"
#include "kernels.hpp"

namespace lgt {

namespace {

template <typename T> struct Ops {
    const void *a, *b;
    void *c;
    int64_t n;
    T s;
};

template <typename T> __device__ __forceinline__ cx<T> ldc(const void *p, int64_t plane, int64_t n, int64_t i)
{
    using V2 = typename std::conditional<std::is_same<T, double>::value, dv2, fv2>::type;
    const V2 v = ((const V2 *)p)[plane * n + i];
    return cx<T>{v.x, v.y};
}
template <typename T> __device__ __forceinline__ void stc(void *p, int64_t plane, int64_t n, int64_t i, cx<T> v)
{
    using V2 = typename std::conditional<std::is_same<T, double>::value, dv2, fv2>::type;
    ((V2 *)p)[plane * n + i] = V2{v.re, v.im};
}

template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> x, cx<T> y)
{
    return cx<T>{x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re};
}
// conj(x) y
template <typename T> __device__ __forceinline__ cx<T> cjmul(cx<T> x, cx<T> y)
{
    return cx<T>{x.re * y.re + x.im * y.im, x.re * y.im - x.im * y.re};
}
// x conj(y)
template <typename T> __device__ __forceinline__ cx<T> mulcj(cx<T> x, cx<T> y)
{
    return cx<T>{x.re * y.re + x.im * y.im, x.im * y.re - x.re * y.im};
}
template <typename T> __device__ __forceinline__ cx<T> cadd(cx<T> x, cx<T> y) { return cx<T>{x.re + y.re, x.im + y.im}; }

// c = A b (66 flop) and c = A^dag b (Eqs (1.1)-(2.3)), A at plane base pa
template <typename T>
__device__ __forceinline__ void matvec(const void *A, int64_t pa, const void *b, int64_t pb, int64_t n, int64_t i,
                                       bool adj, cx<T> c[3])
{
    cx<T> v[3];
#pragma unroll
    for (int j = 0; j < 3; j++) v[j] = ldc<T>(b, pb + j, n, i);
#pragma unroll
    for (int r = 0; r < 3; r++) {
        cx<T> acc{T(0), T(0)};
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const cx<T> m = ldc<T>(A, pa + (adj ? 3 * j + r : 3 * r + j), n, i);
            acc = cadd(acc, adj ? cjmul(m, v[j]) : cmul(m, v[j]));
        }
        c[r] = acc;
    }
}

template <typename T, int R> __global__ __launch_bounds__(kBS) void k_routine(Ops<T> o)
{
    const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (i >= o.n) return;
    const int64_t n = o.n;
    if constexpr (R == LGT_R_ADD_SU3_VECTOR || R == LGT_R_SCALAR_MULT_ADD_SU3_VECTOR) {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            cx<T> x = ldc<T>(o.a, k, n, i), y = ldc<T>(o.b, k, n, i);
            if constexpr (R == LGT_R_SCALAR_MULT_ADD_SU3_VECTOR) {
                y.re *= o.s;
                y.im *= o.s;
            }
            stc<T>(o.c, k, n, i, cadd(x, y));
        }
    } else if constexpr (R == LGT_R_SCALAR_MULT_ADD_SU3_MATRIX) {
#pragma unroll
        for (int k = 0; k < 9; k++) {
            cx<T> x = ldc<T>(o.a, k, n, i), y = ldc<T>(o.b, k, n, i);
            stc<T>(o.c, k, n, i, cx<T>{x.re + o.s * y.re, x.im + o.s * y.im});
        }
    } else if constexpr (R == LGT_R_MULT_SU3_MAT_VEC || R == LGT_R_MULT_ADJ_SU3_MAT_VEC) {
        cx<T> c[3];
        matvec<T>(o.a, 0, o.b, 0, n, i, R == LGT_R_MULT_ADJ_SU3_MAT_VEC, c);
#pragma unroll
        for (int k = 0; k < 3; k++) stc<T>(o.c, k, n, i, c[k]);
    } else if constexpr (R == LGT_R_MULT_ADJ_SU3_MAT_VEC_4DIR || R == LGT_R_MULT_ADJ_SU3_MAT_4VEC) {
        // c_k = B_k^dag a for k = 0..3 (4DIR: a then B4; 4VEC: B4 then a)
        const void *vec = R == LGT_R_MULT_ADJ_SU3_MAT_VEC_4DIR ? o.a : o.b;
        const void *mats = R == LGT_R_MULT_ADJ_SU3_MAT_VEC_4DIR ? o.b : o.a;
#pragma unroll
        for (int d = 0; d < 4; d++) {
            cx<T> c[3];
            matvec<T>(mats, 9 * d, vec, 0, n, i, true, c);
#pragma unroll
            for (int k = 0; k < 3; k++) stc<T>(o.c, 3 * d + k, n, i, c[k]);
        }
    } else if constexpr (R == LGT_R_MULT_SU3_MAT_VEC_SUM_4DIR) {
        cx<T> s[3] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
#pragma unroll
        for (int d = 0; d < 4; d++) {
            cx<T> c[3];
            matvec<T>(o.a, 9 * d, o.b, 3 * d, n, i, false, c);
#pragma unroll
            for (int k = 0; k < 3; k++) s[k] = cadd(s[k], c[k]);
        }
#pragma unroll
        for (int k = 0; k < 3; k++) stc<T>(o.c, k, n, i, s[k]);
    } else if constexpr (R == LGT_R_MULT_SU3_NN || R == LGT_R_MULT_SU3_AN || R == LGT_R_MULT_SU3_NA) {
        // C = op(A) op(B): an = A^dag B, na = A B^dag, nn = A B (198 flop)
        cx<T> A[9], B[9];
#pragma unroll
        for (int k = 0; k < 9; k++) {
            A[k] = ldc<T>(o.a, k, n, i);
            B[k] = ldc<T>(o.b, k, n, i);
        }
#pragma unroll
        for (int r = 0; r < 3; r++) {
#pragma unroll
            for (int q = 0; q < 3; q++) {
                cx<T> acc{T(0), T(0)};
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    if constexpr (R == LGT_R_MULT_SU3_AN) acc = cadd(acc, cjmul(A[3 * k + r], B[3 * k + q]));
                    else if constexpr (R == LGT_R_MULT_SU3_NA) acc = cadd(acc, mulcj(A[3 * r + k], B[3 * q + k]));
                    else acc = cadd(acc, cmul(A[3 * r + k], B[3 * k + q]));
                }
                stc<T>(o.c, 3 * r + q, n, i, acc);
            }
        }
    } else if constexpr (R == LGT_R_SU3_PROJECTOR) {
        cx<T> x[3], y[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            x[k] = ldc<T>(o.a, k, n, i);
            y[k] = ldc<T>(o.b, k, n, i);
        }
#pragma unroll
        for (int r = 0; r < 3; r++) {
#pragma unroll
            for (int q = 0; q < 3; q++) stc<T>(o.c, 3 * r + q, n, i, mulcj(x[r], y[q]));
        }
    } else if constexpr (R == LGT_R_SUB_FOUR_SU3_VECS) {
        // c = a - (b0 + b1 + b2 + b3), c may be a
#pragma unroll
        for (int k = 0; k < 3; k++) {
            cx<T> sum = ldc<T>(o.b, k, n, i);
#pragma unroll
            for (int d = 1; d < 4; d++) sum = cadd(sum, ldc<T>(o.b, 3 * d + k, n, i));
            const cx<T> x = ldc<T>(o.a, k, n, i);
            stc<T>(o.c, k, n, i, cx<T>{x.re - sum.re, x.im - sum.im});
        }
    }
}

template <typename T> hipError_t launch_t(int r, const void *a, const void *b, void *c, int64_t n, double s,
                                          hipStream_t st)
{
    Ops<T> o{a, b, c, n, (T)s};
    const dim3 grid((unsigned)((n + kBS - 1) / kBS)), block(kBS);
    switch (r) {
#define LGT_CASE(R) \
    case R: hipLaunchKernelGGL((k_routine<T, R>), grid, block, 0, st, o); break;
        LGT_CASE(LGT_R_ADD_SU3_VECTOR)
        LGT_CASE(LGT_R_MULT_ADJ_SU3_MAT_VEC)
        LGT_CASE(LGT_R_MULT_ADJ_SU3_MAT_VEC_4DIR)
        LGT_CASE(LGT_R_MULT_ADJ_SU3_MAT_4VEC)
        LGT_CASE(LGT_R_MULT_SU3_AN)
        LGT_CASE(LGT_R_MULT_SU3_NA)
        LGT_CASE(LGT_R_MULT_SU3_NN)
        LGT_CASE(LGT_R_MULT_SU3_MAT_VEC)
        LGT_CASE(LGT_R_MULT_SU3_MAT_VEC_SUM_4DIR)
        LGT_CASE(LGT_R_SCALAR_MULT_ADD_SU3_MATRIX)
        LGT_CASE(LGT_R_SCALAR_MULT_ADD_SU3_VECTOR)
        LGT_CASE(LGT_R_SU3_PROJECTOR)
        LGT_CASE(LGT_R_SUB_FOUR_SU3_VECS)
#undef LGT_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace

hipError_t launch_routine(int routine, bool f64, const void *a, const void *b, void *c, int64_t n, double s,
                          hipStream_t st)
{
    return f64 ? launch_t<double>(routine, a, b, c, n, s, st) : launch_t<float>(routine, a, b, c, n, s, st);
}

} // namespace lgt
