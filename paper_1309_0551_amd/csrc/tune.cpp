// tune.cpp -- choice of the Dslash kernel variant per link format.
//
// The variants differ in how many hops' loads are issued together (8, 2 or
// 1): more loads in flight per thread against fewer registers and more waves
// per SIMD. Which wins depends on the format and the lattice, so it is timed
// on the caller's own link field and kept in the context; with the
// environment variable LGT_TUNE_CACHE naming a file, results persist per
// (device architecture, lattice, format) and later contexts reuse them
// (LGT_TUNE=force re-times).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>

#include "ctx.hpp"

using namespace lgt;

namespace {

const int kVariants[3] = {8, 2, 1};

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

int cache_lookup(const std::string &key)
{
    const char *path = std::getenv("LGT_TUNE_CACHE");
    if (!path) return 0;
    std::ifstream in(path);
    std::string line;
    int found = 0;
    while (std::getline(in, line)) {
        if (line.compare(0, key.size(), key) == 0 && line.size() > key.size() && line[key.size()] == ' ') {
            const int v = std::atoi(line.c_str() + key.size() + 1);
            if (v == 1 || v == 2 || v == 8) found = v; // last entry wins
        }
    }
    return found;
}

void cache_store(const std::string &key, int v, const double t[3])
{
    const char *path = std::getenv("LGT_TUNE_CACHE");
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << key << " " << v << " us:" << t[0] << "," << t[1] << "," << t[2] << "\n";
}

} // namespace

extern "C" {

lgt_status lgt_set_dslash_variant(lgt_ctx *c, int32_t prec, int32_t recon, int32_t hops)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    if (hops != 1 && hops != 2 && hops != 8) return fail(LGT_ERR_ARG, "hops per group must be 1, 2 or 8");
    c->hpi[f] = hops;
    return LGT_OK;
}

lgt_status lgt_get_dslash_variant(lgt_ctx *c, int32_t prec, int32_t recon, int32_t *hops)
{
    clear_error();
    if (!c) return fail(LGT_ERR_ARG, "context is NULL");
    if (!hops) return fail(LGT_ERR_ARG, "hops is NULL");
    Fmt f;
    if (!fmt_of(prec, recon, &f)) return fail(LGT_ERR_UNSUPPORTED, "unsupported link format (%d, %d)", prec, recon);
    *hops = c->hpi[f];
    return LGT_OK;
}

lgt_status lgt_tune_dslash(lgt_ctx *c, const lgt_links *U, double times_us[3])
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
        const int v = cache_lookup(key);
        if (v) {
            c->hpi[f] = v;
            return LGT_OK;
        }
    }
    const size_t vb = (size_t)c->g.Vh * (fmt_is_f64(f) ? 48 : 24);
    void *in = workspace(c, "tune.in", vb);
    void *out = workspace(c, "tune.out", vb);
    if (!in || !out) return fail(LGT_ERR_OOM, "cannot allocate the tuning vectors");
    LGT_HIP(launch_zero(in, vb, c->stream));
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
    a.par = LGT_ODD;
    a.gate = GATE_NONE;
    a.l = site_launch(c->g.Vh);
    double t[3] = {0, 0, 0};
    int best = c->hpi[f];
    double best_t = 1e300;
    const int reps = 10;
    hipError_t e = hipSuccess;
    for (int i = 0; i < 3 && e == hipSuccess; i++) {
        a.hpi = kVariants[i];
        for (int w = 0; w < 2 && e == hipSuccess; w++) e = launch_dslash(f, EPI_PLAIN, a, c->stream);
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; r++) e = launch_dslash(f, EPI_PLAIN, a, c->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        t[i] = 1e3 * ms / reps;
        if (e == hipSuccess && t[i] < best_t) {
            best_t = t[i];
            best = kVariants[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(LGT_ERR_DEVICE, "tuning launch failed: %s", hipGetErrorString(e));
    c->hpi[f] = best;
    cache_store(key, best, t);
    if (times_us)
        for (int i = 0; i < 3; i++) times_us[i] = t[i];
    return LGT_OK;
}

} // extern "C"
