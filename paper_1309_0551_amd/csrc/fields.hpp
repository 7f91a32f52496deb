// fields.hpp -- native structure-of-arrays layouts of link fields and colour
// vectors, and the SU(3) arithmetic of the Dslash.
//
// Links are SU(3) matrices (Sec. 1) with FP32 or FP64 real and imaginary parts
// (Sec. 4), plus BF16 storage. Each format stores, for every (parity, mu), a
// set of planes indexed by the checkerboard index, so that 64 consecutive
// sites of a wavefront read one contiguous, aligned block per load:
//
//   F64 x 18  planes double2[9]   144 B/link   element k = 3*row + col
//   F64 x 12  planes double2[6]    96 B/link   rows 0 and 1
//   F32 x 18  planes float2[9]     72 B/link
//   F32 x 12  planes float4[3]     48 B/link   (U00,U01) (U02,U10) (U11,U12)
//   BF16 x 12 planes [8 x bf16], [4 x bf16]    24 B/link  same element order
//
// Plane (pm, k) of a field with Vh sites per parity starts at element
// ((pm * planes) + k) * Vh with pm = parity*4 + mu (BF16: the 16-byte planes
// of all pm first, then the 8-byte planes).
// 12-real fields rebuild row 2 = conj(row0 x row1), exact for SU(3). Staggered
// phases and boundary signs are never folded into stored links: a sign on a
// stored row would break that identity.
//
// Vectors: planes [3][Vh] of complex (double2 for F64, float2 for F32/BF16).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lgt {

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));
typedef float fv4 __attribute__((ext_vector_type(4)));
typedef uint32_t uv2 __attribute__((ext_vector_type(2)));
typedef uint32_t uv4 __attribute__((ext_vector_type(4)));

template <typename T> struct cx { T re, im; };

// Element i of a plane. The plane base is uniform across the wavefront and the
// index is a 32-bit unsigned value, so the access can use a scalar base with a
// 32-bit vector offset instead of a 64-bit address per lane.
template <bool NT, typename V> __device__ __forceinline__ V ld(const V *plane, unsigned i)
{
    if constexpr (NT) return __builtin_nontemporal_load(plane + i);
    else return plane[i];
}
template <bool NT, typename V> __device__ __forceinline__ void st(V *plane, unsigned i, V v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, plane + i);
    else plane[i] = v;
}

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// Round a double to bfloat16, to nearest even: truncate to float, keep a
// sticky bit in the last float mantissa bit (round to odd), then round the
// float to nearest even at bit 16. Round-to-odd in a format with >= 2 more
// bits makes the second rounding correct.
__device__ __forceinline__ uint32_t bf16_rne(double d)
{
    float f = __double2float_rz(d);
    uint32_t u = __float_as_uint(f);
    if ((double)f != d) u |= 1u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// row 2 of an SU(3) matrix from rows 0 and 1: u2j = conj(u0k u1l - u0l u1k), (j,k,l) cyclic
template <typename T> __device__ __forceinline__ void reconstruct(cx<T> u[9])
{
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const int k = (j + 1) % 3, l = (j + 2) % 3;
        const cx<T> a = u[k], b = u[3 + l], c = u[l], d = u[3 + k];
        const T re = (a.re * b.re - a.im * b.im) - (c.re * d.re - c.im * d.im);
        const T im = (a.re * b.im + a.im * b.re) - (c.re * d.im + c.im * d.re);
        u[6 + j].re = re;
        u[6 + j].im = -im;
    }
}

// The value v of lane K (0..3) of this lane's quad (DPP quad_perm broadcast;
// every lane of the quad must be active).
template <int K> __device__ __forceinline__ uint32_t quad_bcast(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, K * 0x55, 0xF, 0xF, true);
}
template <int K> __device__ __forceinline__ float quad_bcast(float v)
{
    return __uint_as_float(quad_bcast<K>(__float_as_uint(v)));
}

// ---------------------------------------------------------------- links ---
//
// load: the whole link in every lane. load_quad (FP32 / BF16 formats): the
// four lanes q = 0..3 of a quad that all need the same link each load a part
// of it and assemble the rest from their neighbours with quad broadcasts, so
// the vector-memory path returns the link's bytes about once per quad instead
// of four times.

struct LinkF64R18 {
    using real = double;
    static constexpr int bytes = 144;
    static constexpr size_t plane_bytes = 16;
    static constexpr int planes = 9;
    template <bool NT> __device__ static void load(const void *U, size_t Vh, int pm, unsigned cb, cx<double> u[9])
    {
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const dv2 v = ld<NT>((const dv2 *)U + ((size_t)pm * 9 + k) * Vh, cb);
            u[k].re = v.x;
            u[k].im = v.y;
        }
    }
    __device__ static void store(void *U, size_t Vh, int pm, int cb, const double *s)
    {
        dv2 *p = (dv2 *)U + (size_t)pm * 9 * Vh + cb;
        for (int k = 0; k < 9; k++) p[k * Vh] = dv2{s[2 * k], s[2 * k + 1]};
    }
};

struct LinkF64R12 {
    using real = double;
    static constexpr int bytes = 96;
    template <bool NT> __device__ static void load(const void *U, size_t Vh, int pm, unsigned cb, cx<double> u[9])
    {
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const dv2 v = ld<NT>((const dv2 *)U + ((size_t)pm * 6 + k) * Vh, cb);
            u[k].re = v.x;
            u[k].im = v.y;
        }
        reconstruct(u);
    }
    __device__ static void store(void *U, size_t Vh, int pm, int cb, const double *s)
    {
        dv2 *p = (dv2 *)U + (size_t)pm * 6 * Vh + cb;
        for (int k = 0; k < 6; k++) p[k * Vh] = dv2{s[2 * k], s[2 * k + 1]};
    }
};

struct LinkF32R18 {
    using real = float;
    static constexpr int bytes = 72;
    template <bool NT> __device__ static void load(const void *U, size_t Vh, int pm, unsigned cb, cx<float> u[9])
    {
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const fv2 v = ld<NT>((const fv2 *)U + ((size_t)pm * 9 + k) * Vh, cb);
            u[k].re = v.x;
            u[k].im = v.y;
        }
    }
    // planes q and q + 4 from lane q, plane 8 in every lane
    template <bool NT>
    __device__ static void load_quad(const void *U, size_t Vh, int pm, unsigned cb, cx<float> u[9], unsigned q)
    {
        const fv2 *base = (const fv2 *)U + (size_t)pm * 9 * Vh;
        const fv2 a = ld<NT>(base, q * (unsigned)Vh + cb);
        const fv2 b = ld<NT>(base, (q + 4u) * (unsigned)Vh + cb);
        const fv2 c = ld<NT>(base, 8u * (unsigned)Vh + cb);
        u[0] = cx<float>{quad_bcast<0>(a.x), quad_bcast<0>(a.y)};
        u[1] = cx<float>{quad_bcast<1>(a.x), quad_bcast<1>(a.y)};
        u[2] = cx<float>{quad_bcast<2>(a.x), quad_bcast<2>(a.y)};
        u[3] = cx<float>{quad_bcast<3>(a.x), quad_bcast<3>(a.y)};
        u[4] = cx<float>{quad_bcast<0>(b.x), quad_bcast<0>(b.y)};
        u[5] = cx<float>{quad_bcast<1>(b.x), quad_bcast<1>(b.y)};
        u[6] = cx<float>{quad_bcast<2>(b.x), quad_bcast<2>(b.y)};
        u[7] = cx<float>{quad_bcast<3>(b.x), quad_bcast<3>(b.y)};
        u[8] = cx<float>{c.x, c.y};
    }
    __device__ static void store(void *U, size_t Vh, int pm, int cb, const double *s)
    {
        fv2 *p = (fv2 *)U + (size_t)pm * 9 * Vh + cb;
        for (int k = 0; k < 9; k++) p[k * Vh] = fv2{(float)s[2 * k], (float)s[2 * k + 1]};
    }
};

struct LinkF32R12 {
    using real = float;
    static constexpr int bytes = 48;
    template <bool NT> __device__ static void load(const void *U, size_t Vh, int pm, unsigned cb, cx<float> u[9])
    {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const fv4 v = ld<NT>((const fv4 *)U + ((size_t)pm * 3 + k) * Vh, cb);
            u[2 * k].re = v.x;
            u[2 * k].im = v.y;
            u[2 * k + 1].re = v.z;
            u[2 * k + 1].im = v.w;
        }
        reconstruct(u);
    }
    // plane q from lane q < 3 (lane 3 repeats plane 2: the same address)
    template <bool NT>
    __device__ static void load_quad(const void *U, size_t Vh, int pm, unsigned cb, cx<float> u[9], unsigned q)
    {
        const fv4 v = ld<NT>((const fv4 *)U + (size_t)pm * 3 * Vh, (q < 3u ? q : 2u) * (unsigned)Vh + cb);
        u[0] = cx<float>{quad_bcast<0>(v.x), quad_bcast<0>(v.y)};
        u[1] = cx<float>{quad_bcast<0>(v.z), quad_bcast<0>(v.w)};
        u[2] = cx<float>{quad_bcast<1>(v.x), quad_bcast<1>(v.y)};
        u[3] = cx<float>{quad_bcast<1>(v.z), quad_bcast<1>(v.w)};
        u[4] = cx<float>{quad_bcast<2>(v.x), quad_bcast<2>(v.y)};
        u[5] = cx<float>{quad_bcast<2>(v.z), quad_bcast<2>(v.w)};
        reconstruct(u);
    }
    __device__ static void store(void *U, size_t Vh, int pm, int cb, const double *s)
    {
        fv4 *p = (fv4 *)U + (size_t)pm * 3 * Vh + cb;
        for (int k = 0; k < 3; k++)
            p[k * Vh] = fv4{(float)s[4 * k], (float)s[4 * k + 1], (float)s[4 * k + 2], (float)s[4 * k + 3]};
    }
};

struct LinkBF16R12 {
    using real = float;
    static constexpr int bytes = 24;
    template <bool NT> __device__ static void load(const void *U, size_t Vh, int pm, unsigned cb, cx<float> u[9])
    {
        const uv4 a = ld<NT>((const uv4 *)U + (size_t)pm * Vh, cb);
        const uv2 b = ld<NT>((const uv2 *)((const uv4 *)U + 8 * Vh) + (size_t)pm * Vh, cb);
        const uint32_t w[6] = {a.x, a.y, a.z, a.w, b.x, b.y};
#pragma unroll
        for (int k = 0; k < 6; k++) {
            u[k].re = bf16_lo(w[k]);
            u[k].im = bf16_hi(w[k]);
        }
        reconstruct(u);
    }
    // word q of the 16-byte part and word q % 2 of the 8-byte part from lane q
    template <bool NT>
    __device__ static void load_quad(const void *U, size_t Vh, int pm, unsigned cb, cx<float> u[9], unsigned q)
    {
        const uint32_t *a4 = (const uint32_t *)((const uv4 *)U + (size_t)pm * Vh);
        const uint32_t *b2 = (const uint32_t *)((const uv2 *)((const uv4 *)U + 8 * Vh) + (size_t)pm * Vh);
        const uint32_t a = ld<NT>(a4, 4u * cb + q), b = ld<NT>(b2, 2u * cb + (q & 1u));
        const uint32_t w[6] = {quad_bcast<0>(a), quad_bcast<1>(a), quad_bcast<2>(a), quad_bcast<3>(a),
                               quad_bcast<0>(b), quad_bcast<1>(b)};
#pragma unroll
        for (int k = 0; k < 6; k++) {
            u[k].re = bf16_lo(w[k]);
            u[k].im = bf16_hi(w[k]);
        }
        reconstruct(u);
    }
    __device__ static void store(void *U, size_t Vh, int pm, int cb, const double *s)
    {
        uint32_t w[6];
        for (int k = 0; k < 6; k++) w[k] = bf16_rne(s[2 * k]) | (bf16_rne(s[2 * k + 1]) << 16);
        ((uv4 *)U)[(size_t)pm * Vh + cb] = uv4{w[0], w[1], w[2], w[3]};
        ((uv2 *)((uv4 *)U + 8 * Vh))[(size_t)pm * Vh + cb] = uv2{w[4], w[5]};
    }
};

// -------------------------------------------------------------- vectors ---

template <typename T> struct VecFmt;

template <> struct VecFmt<double> {
    using real = double;
    using store_t = dv2;
    static constexpr int bytes = 48;
    template <bool NT> __device__ static void load(const void *v, size_t Vh, unsigned cb, cx<double> o[3])
    {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const dv2 w = ld<NT>((const dv2 *)v + i * Vh, cb);
            o[i].re = w.x;
            o[i].im = w.y;
        }
    }
    template <bool NT> __device__ static void store(void *v, size_t Vh, unsigned cb, const cx<double> o[3])
    {
#pragma unroll
        for (int i = 0; i < 3; i++) st<NT>((dv2 *)v + i * Vh, cb, dv2{o[i].re, o[i].im});
    }
};

template <> struct VecFmt<float> {
    using real = float;
    using store_t = fv2;
    static constexpr int bytes = 24;
    template <bool NT> __device__ static void load(const void *v, size_t Vh, unsigned cb, cx<float> o[3])
    {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const fv2 w = ld<NT>((const fv2 *)v + i * Vh, cb);
            o[i].re = w.x;
            o[i].im = w.y;
        }
    }
    template <bool NT> __device__ static void store(void *v, size_t Vh, unsigned cb, const cx<float> o[3])
    {
#pragma unroll
        for (int i = 0; i < 3; i++) st<NT>((fv2 *)v + i * Vh, cb, fv2{o[i].re, o[i].im});
    }
};

// ------------------------------------------------------------ SU(3) ops ---

// acc += U v  (mult_su3_mat_vec, accumulated)
template <typename T> __device__ __forceinline__ void mv_add(const cx<T> u[9], const cx<T> v[3], cx<T> acc[3])
{
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const cx<T> a = u[3 * i + j];
            acc[i].re = fma(a.re, v[j].re, acc[i].re);
            acc[i].re = fma(-a.im, v[j].im, acc[i].re);
            acc[i].im = fma(a.re, v[j].im, acc[i].im);
            acc[i].im = fma(a.im, v[j].re, acc[i].im);
        }
}

// acc -= U^dag v  (mult_adj_su3_mat_vec, Eqs (1.1)-(2.3), subtracted)
template <typename T> __device__ __forceinline__ void amv_sub(const cx<T> u[9], const cx<T> v[3], cx<T> acc[3])
{
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const cx<T> a = u[3 * j + i];
            acc[i].re = fma(-a.re, v[j].re, acc[i].re);
            acc[i].re = fma(-a.im, v[j].im, acc[i].re);
            acc[i].im = fma(-a.re, v[j].im, acc[i].im);
            acc[i].im = fma(a.im, v[j].re, acc[i].im);
        }
}

template <typename T> __device__ __forceinline__ void negate_if(bool neg, cx<T> v[3])
{
#pragma unroll
    for (int i = 0; i < 3; i++) {
        v[i].re = neg ? -v[i].re : v[i].re;
        v[i].im = neg ? -v[i].im : v[i].im;
    }
}

} // namespace lgt
