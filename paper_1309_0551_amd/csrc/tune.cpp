// tune.cpp -- choice of the Dslash kernel variant per link format.
//
// The variants differ in how many hops' loads are issued together (8, 2 or
// 1: more loads in flight per thread against fewer registers and more waves
// per SIMD), in whether link loads stream past the caches or are cached
// (a link field that fits in the Infinity Cache can then be served from it on
// the next Dslash), and in the workgroup size (256, 128 or 64 sites: a small
// lattice has fewer 256-site workgroups than the chip has CUs). Which wins depends on the format and the lattice, so it is
// timed on the caller's own link field and kept in the context; with the
// environment variable LGT_TUNE_CACHE naming a file, results persist per
// (device architecture, lattice, format) and later contexts reuse them
// (LGT_TUNE=force re-times).
//
// The multi-RHS Dslash is tuned the same way per (format, N): one lane per
// (site, rhs), or groups of four lanes per site (1, 2 or 4 groups, R = N / (4
// groups) right-hand sides per lane) on the VALU or on MFMA -- the tile shape
// trades link-load instructions per site (fewer groups) against registers per
// lane (larger R).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>

#include "batch.hpp"
#include "ctx.hpp"

using namespace lgt;

namespace {

constexpr int kNumVariants = 8;
const int kHops[kNumVariants] = {8, 2, 1, 4, 8, 2, 1, 4};
const int kStream[kNumVariants] = {1, 1, 1, 1, 0, 0, 0, 0};
constexpr int kNumBs = 3;
const int kBsList[kNumBs] = {256, 128, 64};

const char *fmt_name(Fmt f)
{
    switch (f) {
    case F64R18: return "f64r18";
    case F64R12: return "f64r12";
    case F32R18: return "f32r18";
    case F32R12: return "f32r12";
    case BF16R12: return "bf16r12";
    default: return "?";
    }
}

std::string cache_key(lgt_ctx *c, Fmt f)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    std::ostringstream k;
    k << arch << " " << c->geom.L[0] << "x" << c->geom.L[1] << "x" << c->geom.L[2] << "x" << c->geom.L[3] << " "
      << fmt_name(f);
    return k.str();
}

// "<key> <a> <b> ..." with (a, b) accepted by ok(a, b); the last matching line wins
template <class Ok> bool cache_lookup_pair(const std::string &key, int *pa, int *pb, Ok ok)
{
    const char *path = std::getenv("LGT_TUNE_CACHE");
    if (!path) return false;
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        if (line.compare(0, key.size(), key) != 0 || line.size() <= key.size() || line[key.size()] != ' ') continue;
        std::istringstream rest(line.substr(key.size() + 1));
        int a = -1, b = -1;
        rest >> a >> b;
        if (ok(a, b)) {
            *pa = a;
            *pb = b;
            found = true;
        }
    }
    return found;
}

void cache_store_pair(const std::string &key, int a, int b, const double *t, int n)
{
    const char *path = std::getenv("LGT_TUNE_CACHE");
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << key << " " << a << " " << b << " us:";
    for (int i = 0; i < n; i++) out << (i ? "," : "") << t[i];
    out << "\n";
}

// "<key> <hops> <stream> wg<threads> us:..." ; the last matching line wins (a
// line without the workgroup field is a 256-thread choice)
bool cache_lookup(const std::string &key, int *hops, int *stream, int *bs)
{
    const char *path = std::getenv("LGT_TUNE_CACHE");
    if (!path) return false;
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        if (line.compare(0, key.size(), key) != 0 || line.size() <= key.size() || line[key.size()] != ' ') continue;
        std::istringstream rest(line.substr(key.size() + 1));
        int h = -1, st = -1, w = 256;
        std::string tok;
        rest >> h >> st >> tok;
        if (tok.compare(0, 2, "wg") == 0) w = std::atoi(tok.c_str() + 2);
        if ((h == 1 || h == 2 || h == 4 || h == 8) && (st == 0 || st == 1) && dslash_bs_ok(w)) {
            *hops = h;
            *stream = st;
            *bs = w;
            found = true;
        }
    }
    return found;
}

void cache_store(const std::string &key, int hops, int stream, int bs, const double *t, int n)
{
    const char *path = std::getenv("LGT_TUNE_CACHE");
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << key << " " << hops << " " << stream << " wg" << bs << " us:";
    for (int i = 0; i < n; i++) out << (i ? "," : "") << t[i];
    out << "\n";
}

// Runs `step` (one or two launches on s) until kWarmMs of GPU time have
// passed, at most 256 times, before any variant is timed, so that the first
// variants are not timed while the GPU comes out of idle: on all-zero input
// the multi-RHS Dslash (24^3 x 48, 16 right-hand sides) ran its first tens of
// milliseconds after a fifth of a second of idle a fifth slower (89 against
// 74 us); on pseudo-random input no such difference was seen (84-88 us).
constexpr float kWarmMs = 40.f;
template <class Step> hipError_t warm_up(Step step, hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    hipError_t e = hipEventRecord(e0, s);
    for (int round = 0; round < 64 && e == hipSuccess; round++) {
        for (int k = 0; k < 4 && e == hipSuccess; k++) e = step();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms >= kWarmMs) break;
    }
    return e;
}

} // namespace

extern "C" {

lgt_status lgt_set_dslash_variant(lgt_ctx *c, int32_t prec, int32_t recon, int32_t hops, int32_t streaming)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    if (hops != 1 && hops != 2 && hops != 4 && hops != 8)
        return fail(LGT_ERR_ARG, "hops per group must be 1, 2, 4 (LDS-staged) or 8");
    if (streaming != 0 && streaming != 1) return fail(LGT_ERR_ARG, "streaming must be 0 or 1");
    c->hpi[f] = hops;
    c->ntl[f] = streaming;
    return LGT_OK;
}

lgt_status lgt_set_dslash_workgroup(lgt_ctx *c, int32_t prec, int32_t recon, int32_t threads)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    if (!dslash_bs_ok(threads)) return fail(LGT_ERR_ARG, "workgroup size must be 64, 128 or 256");
    c->dbs[f] = threads;
    return LGT_OK;
}

lgt_status lgt_get_dslash_workgroup(lgt_ctx *c, int32_t prec, int32_t recon, int32_t *threads)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    if (!threads) return fail(LGT_ERR_ARG, "output pointer is NULL");
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    *threads = c->dbs[f];
    return LGT_OK;
}

lgt_status lgt_get_dslash_variant(lgt_ctx *c, int32_t prec, int32_t recon, int32_t *hops, int32_t *streaming)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    if (!hops || !streaming) return fail(LGT_ERR_ARG, "output pointer is NULL");
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    *hops = c->hpi[f];
    *streaming = c->ntl[f];
    return LGT_OK;
}

lgt_status lgt_tune_dslash(lgt_ctx *c, const lgt_links *U, double times_us[24])
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    lgt_status st = check_links(U, false, &f);
    if (st != LGT_OK) return st;
    DeviceScope ds(c->device);
    const std::string key = cache_key(c, f);
    const char *force = std::getenv("LGT_TUNE");
    const bool forced = force && std::strcmp(force, "force") == 0;
    if (!forced && !times_us) {
        int h, s, w;
        if (cache_lookup(key, &h, &s, &w)) {
            c->hpi[f] = h;
            c->ntl[f] = s;
            c->dbs[f] = w;
            return LGT_OK;
        }
    }
    const size_t vb = (size_t)c->g.Vh * (fmt_is_f64(f) ? 48 : 24);
    const Launch l = site_launch(c->g.Vh, 64); // the most partial sums of any workgroup size
    void *in = workspace(c, "tune.in", vb);
    void *out = workspace(c, "tune.out", vb);
    void *ap = workspace(c, "tune.ap", vb);
    double *parts = (double *)workspace(c, "tune.partials", sizeof(double) * (size_t)l.nblk_pad);
    CgState *cgs = (CgState *)workspace(c, "tune.state", sizeof(CgState));
    if (!in || !out || !ap || !parts || !cgs) return fail(LGT_ERR_OOM, "cannot allocate the tuning vectors");
    // data like a solver's (on zeros, kernels run faster than in a solve);
    // the zeroed state gives alpha = 0, so r stays as it is
    LGT_HIP(launch_fill_noise(in, vb / (fmt_is_f64(f) ? 8 : 4), fmt_is_f64(f), c->stream));
    LGT_HIP(launch_fill_noise(ap, vb / (fmt_is_f64(f) ? 8 : 4), fmt_is_f64(f), c->stream));
    LGT_HIP(launch_zero(cgs, sizeof(CgState), c->stream));
    hipEvent_t e0, e1;
    LGT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(LGT_ERR_DEVICE, "hipEventCreate failed");
    }
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.U = U->ptr;
    a.in = in;
    a.out = out;
    a.g = c->g;
    a.gate = GATE_NONE;
    a.l = l;
    a.m4 = 0.04;
    a.partials = parts;
    a.st = cgs;
    constexpr int kN = kNumVariants * kNumBs;
    double t[kN] = {};
    double best_t = 1e300;
    const int reps = 5;
    hipError_t e = hipSuccess;
    // the CG's pair: D_oe with the <p, A p> partials, then D_eo with the update
    // of r (alpha from the zeroed state) and its partials (both halves of the
    // link field touched in turn)
    auto pair = [&]() {
        a.par = LGT_ODD;
        a.in = in;
        a.out = out;
        a.aux0 = in;
        hipError_t r = launch_dslash(f, EPI_PAP, a, c->stream);
        if (r != hipSuccess) return r;
        a.par = LGT_EVEN;
        a.in = out;
        a.out = nullptr;
        a.rw = ap;
        return launch_dslash(f, EPI_UPD, a, c->stream);
    };
    // Smaller workgroups only pay where 256-site ones are too few to keep every
    // CU busy; elsewhere they only multiply the CG's per-workgroup partial
    // sums (which the update kernel re-sums in every workgroup), so they are
    // timed only below 1024 workgroups of 256 sites (4 per CU).
    const bool small = site_launch(c->g.Vh).nblk < 1024;
    for (int i = 0; i < kN; i++) t[i] = -1.0;
    a.hpi = kHops[0];
    a.ntl = kStream[0];
    a.l = site_launch(c->g.Vh, kBsList[0]);
    e = warm_up(pair, c->stream, e0, e1);
    for (int i = 0; i < kN && e == hipSuccess; i++) {
        if (kBsList[i / kNumVariants] != 256 && !small) continue;
        a.hpi = kHops[i % kNumVariants];
        a.ntl = kStream[i % kNumVariants];
        a.l = site_launch(c->g.Vh, kBsList[i / kNumVariants]);
        e = pair();
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; r++) e = pair();
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        t[i] = 1e3 * ms / (2 * reps);
        if (e == hipSuccess && t[i] < best_t) best_t = t[i];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(LGT_ERR_DEVICE, "tuning launch failed: %s", hipGetErrorString(e));
    // the first variant in list order within 1 % of the fastest: timing noise
    // alone does not flip the choice between near-equal variants
    int best = 0;
    while (best < kN - 1 && (t[best] < 0.0 || t[best] > 1.01 * best_t)) best++;
    c->hpi[f] = kHops[best % kNumVariants];
    c->ntl[f] = kStream[best % kNumVariants];
    c->dbs[f] = kBsList[best / kNumVariants];
    cache_store(key, c->hpi[f], c->ntl[f], c->dbs[f], t, kN);
    if (times_us)
        for (int i = 0; i < kN; i++) times_us[i] = t[i];
    return LGT_OK;
}

lgt_status lgt_set_dslash_improved_variant(lgt_ctx *c, int32_t prec, int32_t streaming, int32_t threads)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    if (!fmt_of(prec, LGT_R18, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported precision %d", prec);
    if (streaming != 0 && streaming != 1) return fail(LGT_ERR_ARG, "streaming must be 0 or 1");
    if (!dslash_bs_ok(threads)) return fail(LGT_ERR_ARG, "workgroup size must be 64, 128 or 256");
    c->intl[f] = streaming;
    c->ibs[f] = threads;
    return LGT_OK;
}

lgt_status lgt_get_dslash_improved_variant(lgt_ctx *c, int32_t prec, int32_t *streaming, int32_t *threads)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    if (!streaming || !threads) return fail(LGT_ERR_ARG, "output pointer is NULL");
    Fmt f;
    if (!fmt_of(prec, LGT_R18, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported precision %d", prec);
    *streaming = c->intl[f];
    *threads = c->ibs[f];
    return LGT_OK;
}

lgt_status lgt_tune_dslash_improved(lgt_ctx *c, const lgt_links *fat, const lgt_links *naik, double times_us[6])
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    lgt_status st = check_improved(fat, naik, false, &f);
    if (st != LGT_OK) return st;
    DeviceScope ds(c->device);
    const size_t vb = (size_t)c->g.Vh * (fmt_is_f64(f) ? 48 : 24);
    const Launch l64 = site_launch(c->g.Vh, 64); // the most partial sums of any workgroup size
    void *in = workspace(c, "tune.in", vb);
    void *out = workspace(c, "tune.out", vb);
    void *ap = workspace(c, "tune.ap", vb);
    double *parts = (double *)workspace(c, "tune.partials", sizeof(double) * (size_t)l64.nblk_pad);
    CgState *cgs = (CgState *)workspace(c, "tune.state", sizeof(CgState));
    if (!in || !out || !ap || !parts || !cgs) return fail(LGT_ERR_OOM, "cannot allocate the tuning vectors");
    // data like a solver's (timed on zeros, kernels run faster than they do
    // in a solve); the zeroed state gives alpha = 0, so r stays as it is
    LGT_HIP(launch_fill_noise(in, vb / (fmt_is_f64(f) ? 8 : 4), fmt_is_f64(f), c->stream));
    LGT_HIP(launch_fill_noise(ap, vb / (fmt_is_f64(f) ? 8 : 4), fmt_is_f64(f), c->stream));
    LGT_HIP(launch_zero(cgs, sizeof(CgState), c->stream));
    hipEvent_t e0, e1;
    LGT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(LGT_ERR_DEVICE, "hipEventCreate failed");
    }
    DslashArgs a;
    std::memset(&a, 0, sizeof(a));
    a.U = fat->ptr;
    a.U3 = naik->ptr;
    a.g = c->g;
    a.gate = GATE_NONE;
    a.m4 = 0.04;
    a.partials = parts;
    a.st = cgs;
    // the CG's pair, as for the one-link operator
    auto pair = [&]() {
        a.par = LGT_ODD;
        a.in = in;
        a.out = out;
        a.aux0 = in;
        hipError_t r = launch_dslash(f, EPI_PAP, a, c->stream);
        if (r != hipSuccess) return r;
        a.par = LGT_EVEN;
        a.in = out;
        a.out = nullptr;
        a.rw = ap;
        return launch_dslash(f, EPI_UPD, a, c->stream);
    };
    // (streaming, cached) x (256, 128, 64 sites); smaller workgroups only below
    // 1024 workgroups of 256 sites, as for the one-link operator
    constexpr int kN = 2 * kNumBs;
    double t[kN];
    double best_t = 1e300;
    const int reps = 5;
    const bool small = site_launch(c->g.Vh).nblk < 1024;
    for (int i = 0; i < kN; i++) t[i] = -1.0;
    a.ntl = 1;
    a.l = site_launch(c->g.Vh, kBsList[0]);
    hipError_t e = warm_up(pair, c->stream, e0, e1);
    for (int i = 0; i < kN && e == hipSuccess; i++) {
        if (kBsList[i / 2] != 256 && !small) continue;
        a.ntl = 1 - (i & 1);
        a.l = site_launch(c->g.Vh, kBsList[i / 2]);
        e = pair();
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; r++) e = pair();
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        t[i] = 1e3 * ms / (2 * reps);
        if (e == hipSuccess && t[i] < best_t) best_t = t[i];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(LGT_ERR_DEVICE, "tuning launch failed: %s", hipGetErrorString(e));
    int best = 0;
    while (best < kN - 1 && (t[best] < 0.0 || t[best] > 1.01 * best_t)) best++;
    c->intl[f] = 1 - (best & 1);
    c->ibs[f] = kBsList[best / 2];
    if (times_us)
        for (int i = 0; i < kN; i++) times_us[i] = t[i];
    return LGT_OK;
}

} // extern "C"

// ---------------------------------------------------------- multi-RHS ---

namespace {

// lane; VALU and MFMA with 1, 2, 4 groups; the same six LDS-staged
constexpr int kNumMrhs = 13;
const int kMrhsEngine[kNumMrhs] = {MRHS_LANE, MRHS_VALU4, MRHS_VALU4, MRHS_VALU4, MRHS_MFMA, MRHS_MFMA, MRHS_MFMA,
                                   MRHS_VALU4, MRHS_VALU4, MRHS_VALU4, MRHS_MFMA, MRHS_MFMA, MRHS_MFMA};
const int kMrhsGroups[kNumMrhs] = {1, 1, 2, 4, 1, 2, 4, 1, 2, 4, 1, 2, 4};
const int kMrhsStaged[kNumMrhs] = {0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1};
// the tuning cache stores (engine + 10 staged, groups)
constexpr int kStagedCode = 10;

int log2_n(int32_t n)
{
    for (int l = 0; l <= 4; l++)
        if (n == (1 << l)) return l;
    return -1;
}

bool mrhs_variant_runs(Fmt f, const Geom &g, int logN, int v)
{
    if (kMrhsEngine[v] == MRHS_LANE) return true;
    return mrhs_engine_applies(f, logN, g.Vh, kMrhsEngine[v]) && mrhs_groups_valid(logN, kMrhsGroups[v]) &&
           (!kMrhsStaged[v] || mrhs_staging_fits(g, logN, kMrhsGroups[v]));
}

} // namespace

extern "C" {

lgt_status lgt_tune_dslash_mrhs(lgt_ctx *c, const lgt_links *U, int32_t nrhs, double times_us[13])
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    lgt_status st = check_links(U, false, &f);
    if (st != LGT_OK) return st;
    const int logN = log2_n(nrhs);
    if (logN < 0) return fail(LGT_ERR_ARG, "nrhs must be 1, 2, 4, 8 or 16");
    if (!mrhs_size_ok(c->g.Vh)) return fail(LGT_ERR_UNSUPPORTED, "lattice too large for multi-RHS vectors");
    DeviceScope ds(c->device);
    std::ostringstream kk;
    kk << cache_key(c, f) << " mrhs" << nrhs;
    const std::string key = kk.str();
    const char *force = std::getenv("LGT_TUNE");
    const bool forced = force && std::strcmp(force, "force") == 0;
    if (!forced && !times_us) {
        int e, gr;
        auto ok = [&](int a, int b) {
            for (int v = 0; v < kNumMrhs; v++)
                if (kMrhsEngine[v] + kStagedCode * kMrhsStaged[v] == a && kMrhsGroups[v] == b)
                    return mrhs_variant_runs(f, c->g, logN, v);
            return false;
        };
        if (cache_lookup_pair(key, &e, &gr, ok)) {
            c->mrhs_eng[f][logN] = e % kStagedCode;
            c->mrhs_gps[f][logN] = gr;
            c->mrhs_stage[f][logN] = e / kStagedCode;
            return LGT_OK;
        }
    }
    const size_t vb = ((size_t)c->g.Vh << logN) * (fmt_is_f64(f) ? 48 : 24);
    void *in = workspace(c, "tune.mrhs_in", vb);
    void *out = workspace(c, "tune.mrhs_out", vb);
    if (!in || !out) return fail(LGT_ERR_OOM, "cannot allocate the tuning vectors");
    LGT_HIP(launch_fill_noise(in, vb / (fmt_is_f64(f) ? 8 : 4), fmt_is_f64(f), c->stream)); // data like a solver's
    hipEvent_t e0, e1;
    LGT_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(LGT_ERR_DEVICE, "hipEventCreate failed");
    }
    double t[kNumMrhs];
    int best = 0;
    double best_t = 1e300;
    const int reps = 10;
    hipError_t e = hipSuccess;
    for (int v = 0; v < kNumMrhs; v++) t[v] = -1.0;
    for (int v = 0; v < kNumMrhs; v++) {
        if (!mrhs_variant_runs(f, c->g, logN, v)) continue;
        int par = 0;
        e = warm_up(
            [&]() {
                par ^= 1;
                return launch_dslash_mrhs(f, U->ptr, in, out, c->g, par, logN, c->stream, kMrhsEngine[v],
                                          kMrhsGroups[v], kMrhsStaged[v] != 0);
            },
            c->stream, e0, e1);
        break;
    }
    for (int v = 0; v < kNumMrhs && e == hipSuccess; v++) {
        if (!mrhs_variant_runs(f, c->g, logN, v)) continue;
        auto run = [&](int par) {
            return launch_dslash_mrhs(f, U->ptr, in, out, c->g, par, logN, c->stream, kMrhsEngine[v], kMrhsGroups[v],
                                      kMrhsStaged[v] != 0);
        };
        for (int w = 0; w < 2 && e == hipSuccess; w++) e = run(w & 1);
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; r++) e = run(r & 1);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        t[v] = 1e3 * ms / reps;
        if (e == hipSuccess && t[v] < best_t) {
            best_t = t[v];
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(LGT_ERR_DEVICE, "tuning launch failed: %s", hipGetErrorString(e));
    c->mrhs_eng[f][logN] = kMrhsEngine[best];
    c->mrhs_gps[f][logN] = kMrhsGroups[best];
    c->mrhs_stage[f][logN] = kMrhsStaged[best];
    cache_store_pair(key, kMrhsEngine[best] + kStagedCode * kMrhsStaged[best], kMrhsGroups[best], t, kNumMrhs);
    if (times_us)
        for (int v = 0; v < kNumMrhs; v++) times_us[v] = t[v];
    return LGT_OK;
}

} // extern "C"
