// probe.hip -- plain device copy of a known size: the measured HBM ceiling
// next to the 8 TB/s nominal one, and the reference whose FETCH_SIZE /
// WRITE_SIZE counter readings scale the Dslash's counted traffic.
#include <hip/hip_runtime.h>

#include "ctx.hpp"
#include "fields.hpp"

namespace lgt {

__global__ __launch_bounds__(kBS) void k_copy(const uv4 *__restrict__ src, uv4 *__restrict__ dst, size_t n16)
{
    const size_t stride = (size_t)gridDim.x * kBS;
    for (size_t i = (size_t)blockIdx.x * kBS + threadIdx.x; i < n16; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Read-only stream: XOR of the data, stored only if it equals a value no
// real buffer is expected to produce (keeps the loads live at no write cost).
__global__ __launch_bounds__(kBS) void k_read(const uv4 *__restrict__ src, size_t n16, uv4 *__restrict__ sink)
{
    const size_t stride = (size_t)gridDim.x * kBS;
    uv4 acc = uv4{0u, 0u, 0u, 0u};
    for (size_t i = (size_t)blockIdx.x * kBS + threadIdx.x; i < n16; i += stride) acc ^= __builtin_nontemporal_load(src + i);
    if (acc.x == 0x9e3779b9u && acc.y == 0x7f4a7c15u && acc.z == 0xf39cc060u && acc.w == 0x5cedc834u) sink[0] = acc;
}

// The Dslash's link reads alone: one thread per output site of parity par,
// the XCD-remapped block order of the Dslash, its four forward links at the
// site and four backward links at the neighbours x - mu (other parity's
// planes), all loads of the site issued together, streaming or cached; no
// vector gathers, no arithmetic beyond folding the values into one sum, which
// is stored only if it equals a value no real field is expected to produce.
template <class LF, bool NTL>
__global__ __launch_bounds__(kBS) void k_read_links(const void *__restrict__ U, Geom g, int par, Launch l,
                                                    double *__restrict__ sink)
{
    const int blk = xcd_block(blockIdx.x, l.nblk_pad);
    const int cb = blk * kBS + threadIdx.x;
    if (cb >= g.Vh) return;
    int c[4];
    decode(g, par, cb, c);
    using T = typename LF::real;
    T acc = T(0);
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        cx<T> u[9], w[9];
        LF::template load<NTL>(U, (size_t)g.Vh, par * 4 + mu, cb, u);
        LF::template load<NTL>(U, (size_t)g.Vh, (1 - par) * 4 + mu, nbr_bwd(g, c, cb, mu), w);
#pragma unroll
        for (int k = 0; k < 9; k++) acc += (u[k].re + u[k].im) + (w[k].re + w[k].im);
    }
    if (acc == T(1234567.125)) sink[0] = (double)acc;
}

template <class LF>
static void launch_read_links(bool ntl, const void *U, const Geom &g, int par, double *sink, hipStream_t s)
{
    const Launch l = site_launch(g.Vh);
    if (ntl) hipLaunchKernelGGL((k_read_links<LF, true>), dim3(l.nblk_pad), dim3(kBS), 0, s, U, g, par, l, sink);
    else hipLaunchKernelGGL((k_read_links<LF, false>), dim3(l.nblk_pad), dim3(kBS), 0, s, U, g, par, l, sink);
}

} // namespace lgt

using namespace lgt;

extern "C" lgt_status lgt_stream_read_links(lgt_ctx *c, const lgt_links *U, int32_t out_parity, int32_t streaming,
                                            void *sink)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    lgt_status s;
    if ((s = check_links(U, false, &f)) != LGT_OK) return s;
    if ((s = check_ptr(sink, "sink")) != LGT_OK) return s;
    if (out_parity != LGT_EVEN && out_parity != LGT_ODD) return fail(LGT_ERR_ARG, "bad parity %d", out_parity);
    if (streaming != 0 && streaming != 1) return fail(LGT_ERR_ARG, "streaming must be 0 or 1");
    DeviceScope ds(c->device);
    double *sk = (double *)sink;
    switch (f) {
    case F64R18: launch_read_links<LinkF64R18>(streaming, U->ptr, c->g, out_parity, sk, c->stream); break;
    case F64R12: launch_read_links<LinkF64R12>(streaming, U->ptr, c->g, out_parity, sk, c->stream); break;
    case F32R18: launch_read_links<LinkF32R18>(streaming, U->ptr, c->g, out_parity, sk, c->stream); break;
    case F32R12: launch_read_links<LinkF32R12>(streaming, U->ptr, c->g, out_parity, sk, c->stream); break;
    case BF16R12: launch_read_links<LinkBF16R12>(streaming, U->ptr, c->g, out_parity, sk, c->stream); break;
    default: return fail(LGT_ERR_UNSUPPORTED, "unsupported link format");
    }
    LGT_HIP(hipGetLastError());
    return LGT_OK;
}

extern "C" lgt_status lgt_stream_read(lgt_ctx *c, const void *src, size_t bytes, void *sink)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    lgt_status s;
    if ((s = check_ptr(src, "src")) != LGT_OK) return s;
    if ((s = check_ptr(sink, "sink")) != LGT_OK) return s;
    if (bytes % 16) return fail(LGT_ERR_ARG, "bytes must be a multiple of 16");
    const size_t n16 = bytes / 16;
    if (n16 == 0) return LGT_OK;
    DeviceScope ds(c->device);
    size_t blocks = (n16 + kBS - 1) / kBS;
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipLaunchKernelGGL(k_read, dim3((unsigned)blocks), dim3(kBS), 0, c->stream, (const uv4 *)src, n16, (uv4 *)sink);
    LGT_HIP(hipGetLastError());
    return LGT_OK;
}

extern "C" lgt_status lgt_stream_copy(lgt_ctx *c, const void *src, void *dst, size_t bytes)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    lgt_status s;
    if ((s = check_ptr(src, "src")) != LGT_OK) return s;
    if ((s = check_ptr(dst, "dst")) != LGT_OK) return s;
    if (bytes % 16) return fail(LGT_ERR_ARG, "bytes must be a multiple of 16");
    const size_t n16 = bytes / 16;
    if (n16 == 0) return LGT_OK;
    const char *a = (const char *)src;
    const char *b = (const char *)dst;
    if (a < b + bytes && b < a + bytes) return fail(LGT_ERR_ARG, "src and dst overlap");
    DeviceScope ds(c->device);
    size_t blocks = (n16 + kBS - 1) / kBS;
    if (blocks > 256 * 64) blocks = 256 * 64; // 64 workgroups per CU, grid-stride beyond
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(kBS), 0, c->stream, (const uv4 *)src, (uv4 *)dst, n16);
    LGT_HIP(hipGetLastError());
    return LGT_OK;
}
