// abi.cpp -- the extern "C" entry points of lgt.h: argument validation on the
// host, context and workspace management, and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>

#include "ctx.hpp"

namespace lgt {

static thread_local std::string g_last_error;

lgt_status fail(lgt_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

void clear_error() { g_last_error.clear(); }

void *workspace(lgt_ctx *c, const char *name, size_t bytes)
{
    bytes = (bytes + 255) / 256 * 256;
    auto &b = c->ws[name];
    if (b.ptr && b.bytes >= bytes) return b.ptr;
    if (b.ptr) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    if (hipMalloc(&b.ptr, bytes) != hipSuccess) {
        b.ptr = nullptr;
        return nullptr;
    }
    b.bytes = bytes;
    return b.ptr;
}

void *pinned(lgt_ctx *c, size_t bytes)
{
    if (c->pinned && c->pinned_bytes >= bytes) return c->pinned;
    if (c->pinned) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipHostFree(c->pinned);
        c->pinned = nullptr;
        c->pinned_bytes = 0;
    }
    if (hipHostMalloc(&c->pinned, bytes, hipHostMallocDefault) != hipSuccess) {
        c->pinned = nullptr;
        return nullptr;
    }
    c->pinned_bytes = bytes;
    return c->pinned;
}

bool fmt_of(int32_t prec, int32_t recon, Fmt *f)
{
    if (prec == LGT_F64 && recon == LGT_R18) *f = F64R18;
    else if (prec == LGT_F64 && recon == LGT_R12) *f = F64R12;
    else if (prec == LGT_F32 && recon == LGT_R18) *f = F32R18;
    else if (prec == LGT_F32 && recon == LGT_R12) *f = F32R12;
    else if (prec == LGT_BF16 && recon == LGT_R12) *f = BF16R12;
    else return false;
    return true;
}

size_t link_bytes_per_site_dir(Fmt f)
{
    switch (f) {
    case F64R18: return 144;
    case F64R12: return 96;
    case F32R18: return 72;
    case F32R12: return 48;
    case BF16R12: return 24;
    default: return 0;
    }
}

lgt_status check_ptr(const void *p, const char *what)
{
    if (!p) return fail(LGT_ERR_ARG, "%s is NULL", what);
    if (((uintptr_t)p) & 15u) return fail(LGT_ERR_ALIGN, "%s (%p) is not 16-byte aligned", what, p);
    return LGT_OK;
}

lgt_status check_links(const lgt_links *U, bool need_f64, Fmt *f)
{
    if (!U) return fail(LGT_ERR_ARG, "link descriptor is NULL");
    if (!fmt_of(U->prec, U->recon, f))
        return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (prec %d, recon %d)", U->prec, U->recon);
    if (need_f64 && !fmt_is_f64(*f)) return fail(LGT_ERR_ARG, "FP64 links are required here");
    return check_ptr(U->ptr, "link field");
}

lgt_status check_improved(const lgt_links *F, const lgt_links *N, bool need_f64, Fmt *f)
{
    lgt_status s;
    Fmt ff, fn;
    if ((s = check_links(F, need_f64, &ff)) != LGT_OK) return s;
    if ((s = check_links(N, need_f64, &fn)) != LGT_OK) return s;
    if (ff != fn) return fail(LGT_ERR_ARG, "fat and Naik links must have the same format");
    if (ff != F64R18 && ff != F32R18)
        return fail(LGT_ERR_UNSUPPORTED, "the improved operator takes 18-real links (F64 or F32)");
    *f = ff;
    return LGT_OK;
}

static lgt_status geom_check(const lgt_geom *g)
{
    if (!g) return fail(LGT_ERR_ARG, "geometry is NULL");
    int64_t V = 1;
    for (int mu = 0; mu < 4; mu++) {
        if (g->L[mu] < 2 || (g->L[mu] & 1))
            return fail(LGT_ERR_GEOMETRY, "L[%d] = %d must be even and >= 2", mu, g->L[mu]);
        if (g->bc[mu] != 1 && g->bc[mu] != -1)
            return fail(LGT_ERR_GEOMETRY, "bc[%d] = %d must be +1 or -1", mu, g->bc[mu]);
        V *= g->L[mu];
        if (V > ((int64_t)1 << 31)) return fail(LGT_ERR_GEOMETRY, "volume exceeds 2^31 sites");
    }
    return LGT_OK;
}

static Geom make_geom(const lgt_geom *lg)
{
    Geom g;
    for (int mu = 0; mu < 4; mu++) {
        g.L[mu] = lg->L[mu];
        g.bc[mu] = lg->bc[mu];
    }
    g.hx = g.L[0] / 2;
    g.Vh = (int)((int64_t)g.L[0] * g.L[1] * g.L[2] * g.L[3] / 2);
    g.str[0] = 1;
    g.str[1] = g.hx;
    g.str[2] = g.hx * g.L[1];
    g.str[3] = g.hx * g.L[1] * g.L[2];
    return g;
}

lgt_status force_run(lgt_ctx *c, const lgt_links *U, Fmt f, const double *X, double scale, double *G, double *Xn,
                     double *Yn)
{
    LGT_HIP(launch_pack_vec(true, X, Xn, c->g, c->stream));
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.U = U->ptr;
    a.in = Xn;
    a.out = Yn;
    a.g = c->g;
    a.par = LGT_ODD;
    a.gate = GATE_NONE;
    a.l = dslash_launch(c, f);
    a.hpi = c->hpi[f];
    a.ntl = c->ntl[f];
    LGT_HIP(launch_dslash(f, EPI_PLAIN, a, c->stream));
    LGT_HIP(launch_force(Xn, Yn, scale, G, c->g, c->stream));
    return LGT_OK;
}

} // namespace lgt

using namespace lgt;

#define CHECK_CTX(c)                                                  \
    do {                                                              \
        clear_error();                                                \
        if (!(c)) return fail(LGT_ERR_ARG, "context is NULL");        \
    } while (0)

extern "C" {

const char *lgt_status_string(lgt_status s)
{
    switch (s) {
    case LGT_OK: return "ok";
    case LGT_ERR_ARG: return "invalid argument";
    case LGT_ERR_GEOMETRY: return "invalid lattice geometry";
    case LGT_ERR_ALIGN: return "misaligned device pointer";
    case LGT_ERR_DEVICE: return "device or HIP runtime error";
    case LGT_ERR_NOT_CONVERGED: return "solver did not converge";
    case LGT_ERR_NONFINITE: return "non-finite residual or CG breakdown";
    case LGT_ERR_OOM: return "out of device memory";
    case LGT_ERR_UNSUPPORTED: return "unsupported format or device";
    default: return "unknown status";
    }
}

const char *lgt_last_error(void) { return g_last_error.c_str(); }

lgt_status lgt_geom_check(const lgt_geom *g)
{
    clear_error();
    return geom_check(g);
}

lgt_status lgt_links_bytes(const lgt_geom *g, int32_t prec, int32_t recon, size_t *bytes)
{
    clear_error();
    lgt_status s = geom_check(g);
    if (s != LGT_OK) return s;
    if (!bytes) return fail(LGT_ERR_ARG, "bytes is NULL");
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    const int64_t V = (int64_t)g->L[0] * g->L[1] * g->L[2] * g->L[3];
    *bytes = (size_t)V * 4 * link_bytes_per_site_dir(f);
    return LGT_OK;
}

lgt_status lgt_vec_bytes(const lgt_geom *g, int32_t prec, size_t *bytes)
{
    clear_error();
    lgt_status s = geom_check(g);
    if (s != LGT_OK) return s;
    if (!bytes) return fail(LGT_ERR_ARG, "bytes is NULL");
    if (prec != LGT_F64 && prec != LGT_F32 && prec != LGT_BF16) return fail(LGT_ERR_ARG, "bad precision %d", prec);
    const int64_t Vh = (int64_t)g->L[0] * g->L[1] * g->L[2] * g->L[3] / 2;
    *bytes = (size_t)Vh * (prec == LGT_F64 ? 48 : 24);
    return LGT_OK;
}

lgt_status lgt_create(const lgt_geom *g, int32_t device, void *hip_stream, lgt_ctx **out)
{
    clear_error();
    lgt_status s = geom_check(g);
    if (s != LGT_OK) return s;
    if (!out) return fail(LGT_ERR_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(LGT_ERR_DEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(LGT_ERR_DEVICE, "device %d out of range (%d devices)", device, n);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return fail(LGT_ERR_DEVICE, "cannot query device %d", device);
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(LGT_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
    {
        // the device address of the library's fixed scratch array on this
        // device, looked up once (lgt_force_noalloc uses it)
        DeviceScope ds(device);
        if ((s = lgt::scratch_init(device)) != LGT_OK) return s;
    }
    lgt_ctx *c = new (std::nothrow) lgt_ctx();
    if (!c) return fail(LGT_ERR_OOM, "cannot allocate the context");
    c->geom = *g;
    c->g = make_geom(g);
    // FP32 / BF16 link fields: cached loads while the field (mostly) fits in
    // the 256 MB Infinity Cache, which then keeps it from one Dslash to the
    // next; streaming loads for larger fields. Measured on MI355X (CG pair,
    // best variant): cached wins for FP32x12 at 32^4 (201 MB), BF16x12 at
    // 40^4 (246 MB) and FP32x18 at 32^4 (302 MB); streaming for FP32x12 at
    // 40^4 (491 MB), FP32x18 at 40^4 (737 MB) and BF16x12 at 48^4 (510 MB).
    const size_t V = 2 * (size_t)c->g.Vh;
    for (int f = F32R18; f <= BF16R12; f++)
        c->ntl[f] = V * 4 * link_bytes_per_site_dir((Fmt)f) > kMallBytes * 3 / 2;
    // FP64 fields that fit in half the Infinity Cache (16^4: 37.7 MB) take the
    // fully unrolled kernel with cached link loads (measured at 16^4 FP64x18:
    // 7.5 us against 12.5 us for 2 hops streaming); larger FP64 fields keep 2
    // hops and streaming loads (24^3x48, 382 MB: 73.6 us against 80.0 cached).
    for (int f = F64R18; f <= F64R12; f++)
        if (V * 4 * link_bytes_per_site_dir((Fmt)f) <= kMallBytes / 2) {
            c->hpi[f] = 8;
            c->ntl[f] = 0;
        }
    // the improved operator reads two 18-real fields
    for (int f = 0; f < FMT_COUNT; f++) c->intl[f] = 2 * V * 4 * link_bytes_per_site_dir((Fmt)f) > kMallBytes * 3 / 2;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return LGT_OK;
}

lgt_status lgt_destroy(lgt_ctx *c)
{
    CHECK_CTX(c);
    {
        DeviceScope ds(c->device);
        (void)hipStreamSynchronize(c->stream);
        if (c->aux) {
            (void)hipStreamSynchronize(c->aux);
            (void)hipStreamDestroy(c->aux);
        }
        for (auto &kv : c->ws)
            if (kv.second.ptr) (void)hipFree(kv.second.ptr);
        if (c->pinned) (void)hipHostFree(c->pinned);
    }
    delete c;
    return LGT_OK;
}

lgt_status lgt_cg_profile(lgt_ctx *c, double ms[4], int32_t *n)
{
    CHECK_CTX(c);
    if (!ms || !n) return fail(LGT_ERR_ARG, "output pointer is NULL");
    for (int k = 0; k < 4; k++) ms[k] = c->cg_prof_ms[k];
    *n = c->cg_prof_n;
    return LGT_OK;
}

lgt_status lgt_cg_dslash_profile(lgt_ctx *c, double ms[4], int32_t n[4])
{
    CHECK_CTX(c);
    if (!ms || !n) return fail(LGT_ERR_ARG, "output pointer is NULL");
    for (int k = 0; k < 4; k++) {
        ms[k] = c->cg_dsl_ms[k];
        n[k] = c->cg_dsl_n[k];
    }
    return LGT_OK;
}

lgt_status lgt_set_timing(lgt_ctx *c, int32_t every)
{
    CHECK_CTX(c);
    if (every < 0) return fail(LGT_ERR_ARG, "timing interval must be >= 0");
    c->timing = every;
    return LGT_OK;
}

lgt_status lgt_index_maps(lgt_ctx *c, int32_t *lex_of_eo, int32_t *nbr)
{
    CHECK_CTX(c);
    lgt_status s;
    if ((s = check_ptr(lex_of_eo, "lex_of_eo")) != LGT_OK) return s;
    if ((s = check_ptr(nbr, "nbr")) != LGT_OK) return s;
    DeviceScope ds(c->device);
    LGT_HIP(launch_index_maps(lex_of_eo, nbr, c->g, c->stream));
    return LGT_OK;
}

lgt_status lgt_pack_links(lgt_ctx *c, const double *Uc, int32_t prec, int32_t recon, void *Up)
{
    CHECK_CTX(c);
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    lgt_status s;
    if ((s = check_ptr(Uc, "U_canon")) != LGT_OK) return s;
    if ((s = check_ptr(Up, "U_packed")) != LGT_OK) return s;
    DeviceScope ds(c->device);
    LGT_HIP(launch_pack_links(f, Uc, Up, c->g, c->stream));
    return LGT_OK;
}

lgt_status lgt_unpack_links(lgt_ctx *c, const void *Up, int32_t prec, int32_t recon, double *Uc)
{
    CHECK_CTX(c);
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    lgt_status s;
    if ((s = check_ptr(Up, "U_packed")) != LGT_OK) return s;
    if ((s = check_ptr(Uc, "U_canon")) != LGT_OK) return s;
    DeviceScope ds(c->device);
    LGT_HIP(launch_unpack_links(f, Up, Uc, c->g, c->stream));
    return LGT_OK;
}

static lgt_status vec_prec_ok(int32_t prec, bool *f64)
{
    if (prec == LGT_F64) *f64 = true;
    else if (prec == LGT_F32 || prec == LGT_BF16) *f64 = false;
    else return fail(LGT_ERR_ARG, "bad precision %d", prec);
    return LGT_OK;
}

lgt_status lgt_pack_vec(lgt_ctx *c, int32_t prec, const double *src, void *dst)
{
    CHECK_CTX(c);
    bool f64;
    lgt_status s;
    if ((s = vec_prec_ok(prec, &f64)) != LGT_OK) return s;
    if ((s = check_ptr(src, "src")) != LGT_OK) return s;
    if ((s = check_ptr(dst, "dst")) != LGT_OK) return s;
    DeviceScope ds(c->device);
    LGT_HIP(launch_pack_vec(f64, src, dst, c->g, c->stream));
    return LGT_OK;
}

lgt_status lgt_unpack_vec(lgt_ctx *c, int32_t prec, const void *src, double *dst)
{
    CHECK_CTX(c);
    bool f64;
    lgt_status s;
    if ((s = vec_prec_ok(prec, &f64)) != LGT_OK) return s;
    if ((s = check_ptr(src, "src")) != LGT_OK) return s;
    if ((s = check_ptr(dst, "dst")) != LGT_OK) return s;
    DeviceScope ds(c->device);
    LGT_HIP(launch_unpack_vec(f64, src, dst, c->g, c->stream));
    return LGT_OK;
}

lgt_status lgt_dslash(lgt_ctx *c, const lgt_links *U, int32_t out_parity, const void *in, void *out)
{
    CHECK_CTX(c);
    Fmt f;
    lgt_status s;
    if ((s = check_links(U, false, &f)) != LGT_OK) return s;
    if (out_parity != LGT_EVEN && out_parity != LGT_ODD) return fail(LGT_ERR_ARG, "bad parity %d", out_parity);
    if ((s = check_ptr(in, "in")) != LGT_OK) return s;
    if ((s = check_ptr(out, "out")) != LGT_OK) return s;
    if (in == out) return fail(LGT_ERR_ARG, "in and out alias");
    DeviceScope ds(c->device);
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.U = U->ptr;
    a.in = in;
    a.out = out;
    a.g = c->g;
    a.par = out_parity;
    a.gate = GATE_NONE;
    a.l = dslash_launch(c, f);
    a.hpi = c->hpi[f];
    a.ntl = c->ntl[f];
    LGT_HIP(launch_dslash(f, EPI_PLAIN, a, c->stream));
    return LGT_OK;
}

lgt_status lgt_apply_normal(lgt_ctx *c, const lgt_links *U, double mass, const void *in, void *out, double *pAp)
{
    CHECK_CTX(c);
    Fmt f;
    lgt_status s;
    if ((s = check_links(U, false, &f)) != LGT_OK) return s;
    if (!(mass >= 0.0) || !std::isfinite(mass)) return fail(LGT_ERR_ARG, "mass must be finite and >= 0");
    if ((s = check_ptr(in, "in")) != LGT_OK) return s;
    if ((s = check_ptr(out, "out")) != LGT_OK) return s;
    if (in == out) return fail(LGT_ERR_ARG, "in and out alias");
    DeviceScope ds(c->device);
    const size_t vb = (size_t)c->g.Vh * (fmt_is_f64(f) ? 48 : 24);
    const Launch l = dslash_launch(c, f);
    void *t = workspace(c, "apply.t", vb);
    double *parts = (double *)workspace(c, "apply.partials", sizeof(double) * (size_t)l.nblk_pad);
    double *host = pAp ? (double *)pinned(c, sizeof(double) * (size_t)l.nblk_pad) : nullptr;
    if (!t || !parts || (pAp && !host)) return fail(LGT_ERR_OOM, "cannot allocate the workspace");
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.U = U->ptr;
    a.g = c->g;
    a.gate = GATE_NONE;
    a.l = l;
    a.hpi = c->hpi[f];
    a.ntl = c->ntl[f];
    a.par = LGT_ODD; // t = D_oe in
    a.in = in;
    a.out = t;
    LGT_HIP(launch_dslash(f, EPI_PLAIN, a, c->stream));
    a.par = LGT_EVEN; // out = 4m^2 in - D_eo t, one partial <in, out> per workgroup
    a.in = t;
    a.out = out;
    a.aux0 = in;
    a.m4 = 4.0 * mass * mass;
    a.partials = parts;
    LGT_HIP(launch_dslash(f, EPI_A, a, c->stream));
    if (pAp) {
        LGT_HIP(hipMemcpyAsync(host, parts, sizeof(double) * (size_t)l.nblk_pad, hipMemcpyDeviceToHost, c->stream));
        LGT_HIP(hipStreamSynchronize(c->stream));
        double sum = 0.0;
        for (int i = 0; i < l.nblk; i++) sum += host[i]; // slots past nblk hold zeros
        *pAp = sum;
    }
    return LGT_OK;
}

namespace {

lgt_status check_cg_params(const lgt_cg_params *p)
{
    if (!p) return fail(LGT_ERR_ARG, "params is NULL");
    if (!(p->mass > 0.0)) return fail(LGT_ERR_ARG, "mass must be > 0");
    if (!(p->tol > 0.0)) return fail(LGT_ERR_ARG, "tol must be > 0");
    if (p->max_iter <= 0) return fail(LGT_ERR_ARG, "max_iter must be > 0");
    if (p->scheme < LGT_CG_FP64 || p->scheme > LGT_CG_REFINE) return fail(LGT_ERR_ARG, "bad scheme %d", p->scheme);
    if (p->scheme == LGT_CG_RELIABLE && p->ru_interval <= 0) return fail(LGT_ERR_ARG, "ru_interval must be > 0");
    if (p->scheme == LGT_CG_REFINE && !(p->inner_tol > 0.0 && p->inner_tol < 1.0))
        return fail(LGT_ERR_ARG, "inner_tol must be in (0, 1) for refinement");
    if (p->scheme != LGT_CG_REFINE && (p->inner_tol < 0.0 || p->inner_tol > 1.0))
        return fail(LGT_ERR_ARG, "inner_tol must be in [0, 1]");
    if (p->check_interval < 0) return fail(LGT_ERR_ARG, "check_interval must be >= 0");
    return LGT_OK;
}

// improved operator: fat and Naik fields in one 18-real format
} // namespace

lgt_status lgt_cg_solve(lgt_ctx *c, const lgt_links *Uhi, const lgt_links *Ulo, const lgt_cg_params *p,
                        const double *b, double *x, lgt_cg_result *res)
{
    CHECK_CTX(c);
    lgt_status s;
    if ((s = check_cg_params(p)) != LGT_OK) return s;
    if ((s = check_ptr(b, "b")) != LGT_OK) return s;
    if ((s = check_ptr(x, "x")) != LGT_OK) return s;
    DeviceScope ds(c->device);
    return cg_solve(c, Uhi, Ulo, p, b, x, res);
}

lgt_status lgt_dslash_improved(lgt_ctx *c, const lgt_links *fat, const lgt_links *naik, int32_t out_parity,
                               const void *in, void *out)
{
    CHECK_CTX(c);
    Fmt f;
    lgt_status s;
    if ((s = check_improved(fat, naik, false, &f)) != LGT_OK) return s;
    if (out_parity != LGT_EVEN && out_parity != LGT_ODD) return fail(LGT_ERR_ARG, "bad parity %d", out_parity);
    if ((s = check_ptr(in, "in")) != LGT_OK) return s;
    if ((s = check_ptr(out, "out")) != LGT_OK) return s;
    if (in == out) return fail(LGT_ERR_ARG, "in and out alias");
    DeviceScope ds(c->device);
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.U = fat->ptr;
    a.U3 = naik->ptr;
    a.in = in;
    a.out = out;
    a.g = c->g;
    a.par = out_parity;
    a.gate = GATE_NONE;
    a.l = dslash_launch_improved(c, f);
    a.ntl = c->intl[f];
    LGT_HIP(launch_dslash(f, EPI_PLAIN, a, c->stream));
    return LGT_OK;
}

lgt_status lgt_cg_solve_improved(lgt_ctx *c, const lgt_links *fat_hi, const lgt_links *naik_hi,
                                 const lgt_links *fat_lo, const lgt_links *naik_lo, const lgt_cg_params *p,
                                 const double *b, double *x, lgt_cg_result *res)
{
    CHECK_CTX(c);
    lgt_status s;
    if ((s = check_cg_params(p)) != LGT_OK) return s;
    Fmt f;
    if ((s = check_improved(fat_hi, naik_hi, true, &f)) != LGT_OK) return s;
    if (p->scheme != LGT_CG_FP64) {
        if ((s = check_improved(fat_lo, naik_lo, false, &f)) != LGT_OK) return s;
        if (f != F32R18) return fail(LGT_ERR_ARG, "the inner links of a mixed scheme must be F32 x 18");
    }
    if ((s = check_ptr(b, "b")) != LGT_OK) return s;
    if ((s = check_ptr(x, "x")) != LGT_OK) return s;
    DeviceScope ds(c->device);
    return cg_solve(c, fat_hi, fat_lo, p, b, x, res, naik_hi, naik_lo);
}

lgt_status lgt_routine(lgt_ctx *c, int32_t routine, int32_t prec, int64_t n, const void *a, const void *b,
                       void *out, double s)
{
    CHECK_CTX(c);
    switch (routine) {
    case LGT_R_ADD_SU3_VECTOR: case LGT_R_MULT_ADJ_SU3_MAT_VEC: case LGT_R_MULT_ADJ_SU3_MAT_VEC_4DIR:
    case LGT_R_MULT_ADJ_SU3_MAT_4VEC: case LGT_R_MULT_SU3_AN: case LGT_R_MULT_SU3_NA: case LGT_R_MULT_SU3_NN:
    case LGT_R_MULT_SU3_MAT_VEC: case LGT_R_MULT_SU3_MAT_VEC_SUM_4DIR: case LGT_R_SCALAR_MULT_ADD_SU3_MATRIX:
    case LGT_R_SCALAR_MULT_ADD_SU3_VECTOR: case LGT_R_SU3_PROJECTOR: case LGT_R_SUB_FOUR_SU3_VECS: break;
    case 2: case 7: return fail(LGT_ERR_UNSUPPORTED, "routine %d works on Wilson half-vectors", routine);
    default: return fail(LGT_ERR_ARG, "unknown routine %d", routine);
    }
    if (prec != LGT_F64 && prec != LGT_F32) return fail(LGT_ERR_ARG, "precision must be LGT_F64 or LGT_F32");
    if (n < 0 || n > ((int64_t)1 << 40)) return fail(LGT_ERR_ARG, "bad n %lld", (long long)n);
    if (n == 0) return LGT_OK;
    lgt_status st;
    if ((st = check_ptr(a, "a")) != LGT_OK) return st;
    if ((st = check_ptr(b, "b")) != LGT_OK) return st;
    if ((st = check_ptr(out, "c")) != LGT_OK) return st;
    if (!std::isfinite(s)) return fail(LGT_ERR_ARG, "s must be finite");
    DeviceScope ds(c->device);
    LGT_HIP(launch_routine(routine, prec == LGT_F64, a, b, out, n, s, c->stream));
    return LGT_OK;
}

lgt_status lgt_cdot(lgt_ctx *c, int64_t n, const double *a, const double *b, double out[2])
{
    CHECK_CTX(c);
    if (n < 0) return fail(LGT_ERR_ARG, "n must be >= 0");
    if (!out) return fail(LGT_ERR_ARG, "out is NULL");
    lgt_status s;
    if ((s = check_ptr(a, "a")) != LGT_OK) return s;
    if ((s = check_ptr(b, "b")) != LGT_OK) return s;
    DeviceScope ds(c->device);
    double *part = (double *)workspace(c, "dot.partials", 2 * 1024 * sizeof(double));
    double *res = (double *)workspace(c, "dot.result", 2 * sizeof(double) + sizeof(unsigned int) * 4);
    double *host = (double *)pinned(c, 3 * sizeof(CgState));
    if (!part || !res || !host) return fail(LGT_ERR_OOM, "cannot allocate the reduction workspace");


    LGT_HIP(launch_cdot(n, a, b, part, res, c->stream));
    LGT_HIP(hipMemcpyAsync(host, res, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LGT_HIP(hipStreamSynchronize(c->stream));
    out[0] = host[0];
    out[1] = host[1];
    return LGT_OK;
}

lgt_status lgt_force(lgt_ctx *c, const lgt_links *U, const double *X, double scale, double *G)
{
    CHECK_CTX(c);
    Fmt f;
    lgt_status s;
    if ((s = check_links(U, true, &f)) != LGT_OK) return s;
    if ((s = check_ptr(X, "X")) != LGT_OK) return s;
    if ((s = check_ptr(G, "G")) != LGT_OK) return s;
    if (!std::isfinite(scale)) return fail(LGT_ERR_ARG, "scale must be finite");
    DeviceScope ds(c->device);
    const size_t v64 = (size_t)c->g.Vh * 48;
    double *Xn = (double *)workspace(c, "force.X", v64);
    double *Yn = (double *)workspace(c, "force.Y", v64);
    if (!Xn || !Yn) return fail(LGT_ERR_OOM, "cannot allocate the force workspace");
    return lgt::force_run(c, U, f, X, scale, G, Xn, Yn);
}

lgt_status lgt_action_phi_grad(lgt_ctx *c, const double *X, double scale, double *gphi)
{
    CHECK_CTX(c);
    lgt_status s;
    if ((s = check_ptr(X, "X")) != LGT_OK) return s;
    if ((s = check_ptr(gphi, "gphi")) != LGT_OK) return s;
    if (!std::isfinite(scale)) return fail(LGT_ERR_ARG, "scale must be finite");
    DeviceScope ds(c->device);
    LGT_HIP(launch_phi_grad(X, scale, gphi, c->g, c->stream));
    return LGT_OK;
}

lgt_status lgt_force_improved(lgt_ctx *c, const lgt_links *fat, const lgt_links *naik, const double *X, double scale,
                              double *G_fat, double *G_naik)
{
    CHECK_CTX(c);
    Fmt f;
    lgt_status s;
    if ((s = check_improved(fat, naik, true, &f)) != LGT_OK) return s;
    if ((s = check_ptr(X, "X")) != LGT_OK) return s;
    if ((s = check_ptr(G_fat, "G_fat")) != LGT_OK) return s;
    if ((s = check_ptr(G_naik, "G_naik")) != LGT_OK) return s;
    if (G_fat == G_naik) return fail(LGT_ERR_ARG, "G_fat and G_naik alias");
    if (!std::isfinite(scale)) return fail(LGT_ERR_ARG, "scale must be finite");
    DeviceScope ds(c->device);
    const size_t v64 = (size_t)c->g.Vh * 48;
    double *Xn = (double *)workspace(c, "force.X", v64);
    double *Yn = (double *)workspace(c, "force.Y", v64);
    if (!Xn || !Yn) return fail(LGT_ERR_OOM, "cannot allocate the force workspace");
    LGT_HIP(launch_pack_vec(true, X, Xn, c->g, c->stream));
    DslashArgs a; // Y = D_oe X with the one-link and three-link hops
    std::memset(&a, 0, sizeof(a));
    a.U = fat->ptr;
    a.U3 = naik->ptr;
    a.in = Xn;
    a.out = Yn;
    a.g = c->g;
    a.par = LGT_ODD;
    a.gate = GATE_NONE;
    a.l = dslash_launch_improved(c, f);
    a.ntl = c->intl[f];
    LGT_HIP(launch_dslash(f, EPI_PLAIN, a, c->stream));
    LGT_HIP(launch_force(Xn, Yn, scale, G_fat, c->g, c->stream, false));
    LGT_HIP(launch_force(Xn, Yn, scale, G_naik, c->g, c->stream, true));
    return LGT_OK;
}

} // extern "C"
