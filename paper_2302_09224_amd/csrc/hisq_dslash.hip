// hisq_dslash.hip -- dispatch of the Dslash launches on the precision triplet
// gauge/fermion/compute (Sec. 4) and the launch-shape autotuner.  The kernels
// are instantiated in hisq_dslash_t_*.hip (one translation unit per triplet).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "hisq_internal.h"

namespace hisq {

#define HISQ_DECL_TRIPLET(NAME)                                                                              \
    hipError_t dslash_launch_##NAME(const DslashArgs &a, int rhs0, const DslashTile &t, hipStream_t st, int *nb); \
    hipError_t dslash_multi_##NAME(const MultiArgs &m, int long_recon, hipStream_t st);
HISQ_DECL_TRIPLET(double)
HISQ_DECL_TRIPLET(single)
HISQ_DECL_TRIPLET(half)
HISQ_DECL_TRIPLET(int20)
HISQ_DECL_TRIPLET(int30)
HISQ_DECL_TRIPLET(int30_fp32)
HISQ_DECL_TRIPLET(int24)
HISQ_DECL_TRIPLET(sx24)
HISQ_DECL_TRIPLET(sx24_int30)

namespace {

inline int triplet_key(const hisq_fmt &f) { return f.gauge * 100 + f.spinor * 10 + (f.compute == 64 ? 1 : 0); }

hipError_t launch_one(const DslashArgs &a, const hisq_fmt &f, int rhs0, const DslashTile &t, hipStream_t st, int *nb) {
    switch (triplet_key(f)) {
    case GF_F64 * 100 + SF_F64 * 10 + 1: return dslash_launch_double(a, rhs0, t, st, nb);
    case GF_F32 * 100 + SF_F32 * 10 + 0: return dslash_launch_single(a, rhs0, t, st, nb);
    case GF_FIX16 * 100 + SF_HALF16 * 10 + 0: return dslash_launch_half(a, rhs0, t, st, nb);
    case GF_FIX16 * 100 + SF_INT20 * 10 + 0: return dslash_launch_int20(a, rhs0, t, st, nb);
    case GF_FIX32 * 100 + SF_INT30 * 10 + 1: return dslash_launch_int30(a, rhs0, t, st, nb);
    case GF_FIX32 * 100 + SF_INT30 * 10 + 0: return dslash_launch_int30_fp32(a, rhs0, t, st, nb);
    case GF_FIX32 * 100 + SF_INT24 * 10 + 0: return dslash_launch_int24(a, rhs0, t, st, nb);
    case GF_SX24 * 100 + SF_INT24 * 10 + 0: return dslash_launch_sx24(a, rhs0, t, st, nb);
    case GF_SX24 * 100 + SF_INT30 * 10 + 1: return dslash_launch_sx24_int30(a, rhs0, t, st, nb);
    default: return hipErrorInvalidValue;
    }
}

// triplet + long-link storage, X, Y, Z, T, rhs block, fused reduction (0 or 1)
typedef std::tuple<int, int, int, int, int, int, int> TuneKey;

inline int tune_id(const hisq_fmt &f, int long_recon) {
    return triplet_key(f) * 100 + (long_recon == 12 ? 12 : long_recon == 8 ? 8 : 18);
}
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<DslashTile, float>> g_tuned;

bool tuning_enabled() {
    const char *e = getenv("HISQ_TUNE");
    return !(e && e[0] == '0');
}

// a launch shape the kernels are instantiated for, for a block of c right-hand sides
bool shape_ok(const hisq_fmt &f, int c, const DslashTile &t) {
    bool ok = t.nr >= 1 && t.rg >= 1 && t.nr * t.rg == c && (t.nr & (t.nr - 1)) == 0 && (t.rg & (t.rg - 1)) == 0;
    ok = ok && (t.block == 128 || t.block == 256) && t.grid >= 0 && t.grid % 8 == 0 && t.sweep >= 0 && t.sweep <= 2;
    const bool mfma = t.stage == 5 && t.rg == 4 && t.nr <= 4 && f.compute == 32;   // the matrix-core path
    return ok && (mfma || (t.nr == 1 ? (t.stage == 1 || t.stage == 2 || t.stage == 4 || t.stage == 8 ||
                                        t.stage == -1 || t.stage == -2)
                                     : (t.stage == 1 || (t.stage == -1 && t.nr <= 8))));
}

// ---------------------------------------------------------------------------
// Tune cache files.  One text line per shape key:
//   hisq-tune <version> <arch> <hip runtime> <triplet*100+recon> X Y Z T <rhs block> <fused> :
//       nr rg stage block grid sweep <microseconds>
// Lines of another format version, device architecture or HIP runtime
// version are skipped on reading (their timings say nothing about this one).
// ---------------------------------------------------------------------------
constexpr int kTuneFileVersion = 1;

// "gfx950 <runtime version>" of the current device, or "" without one
std::string device_tag() {
    int dev = 0, rv = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        hipRuntimeGetVersion(&rv) != hipSuccess) {
        (void)hipGetLastError();
        return std::string();
    }
    std::string arch(prop.gcnArchName);
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return arch + " " + std::to_string(rv);
}

std::string tune_line(const std::string &tag, const TuneKey &k, const DslashTile &t, float ms) {
    char line[320];
    snprintf(line, sizeof(line), "hisq-tune %d %s %d %d %d %d %d %d %d : %d %d %d %d %d %d %.3f\n", kTuneFileVersion,
             tag.c_str(), std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
             std::get<5>(k), std::get<6>(k), t.nr, t.rg, t.stage, t.block, t.grid, t.sweep, ms * 1e3);
    return std::string(line);
}

// Parse `path` into entries for device `tag` (g_tune_mu held by the caller when
// `apply`); `replace`: a line replaces the table's entry of the same key, else
// only keys without an entry are filled.  Returns HISQ_EIO for an unreadable
// file or a malformed line.
hisq_status read_tune_file(const char *path, const std::string &tag, bool apply, bool replace, int *nloaded) {
    FILE *fp = fopen(path, "r");
    if (!fp) return set_error(HISQ_EIO, "tune cache %s: cannot open", path);
    std::vector<std::pair<TuneKey, DslashTile>> got;
    char line[512];
    int lineno = 0;
    hisq_status st = HISQ_OK;
    while (fgets(line, sizeof(line), fp)) {
        lineno++;
        if (line[0] == '\n' || line[0] == '#') continue;
        int ver = 0, rv = 0, tid = 0, X, Y, Z, T, c, red, nr, rg, stage, block, grid, sweep;
        char arch[64];
        float us = 0.f;
        const int n = sscanf(line, "hisq-tune %d %63s %d %d %d %d %d %d %d %d : %d %d %d %d %d %d %f", &ver, arch, &rv,
                             &tid, &X, &Y, &Z, &T, &c, &red, &nr, &rg, &stage, &block, &grid, &sweep, &us);
        if (n != 17) {
            st = set_error(HISQ_EIO, "tune cache %s: malformed line %d", path, lineno);
            break;
        }
        if (ver != kTuneFileVersion || tag != std::string(arch) + " " + std::to_string(rv)) continue;
        const hisq_fmt f{tid / 10000, (tid / 1000) % 10, (tid / 100) % 10 ? 64 : 32};
        const int recon = tid % 100;
        const int dims[4] = {X, Y, Z, T};
        const DslashTile t{nr, rg, stage, block, grid, sweep};
        const bool pow2 = c >= 1 && c <= 16 && (c & (c - 1)) == 0;
        if (!dims_ok(dims) || !triplet_ok(f) || (recon != 8 && recon != 12 && recon != 18) ||
            !recon_ok(f, recon, c > 1) || !pow2 || (red != 0 && red != 1) ||
            (c > 1 && !has_batched_form(f)) || !shape_ok(f, c, t)) {
            st = set_error(HISQ_EIO, "tune cache %s: line %d names an unsupported key or shape", path, lineno);
            break;
        }
        got.emplace_back(TuneKey{tid, X, Y, Z, T, c, red}, t);
    }
    fclose(fp);
    if (st != HISQ_OK) return st;
    if (apply)
        for (const auto &e : got) {
            if (replace)
                g_tuned[e.first] = std::make_pair(e.second, -1.f);
            else
                g_tuned.emplace(e.first, std::make_pair(e.second, -1.f));
        }
    if (nloaded) *nloaded = (int)got.size();
    return HISQ_OK;
}

// HISQ_TUNE_CACHE=<path>: shapes read from the file at the first lookup of the
// process, and every shape tuned afterwards appended to it
const char *cache_path() {
    const char *p = getenv("HISQ_TUNE_CACHE");
    return (p && p[0]) ? p : nullptr;
}
bool g_cache_read = false;

void cache_read_once() {
    if (g_cache_read) return;
    g_cache_read = true;
    const char *path = cache_path();
    if (!path) return;
    const std::string tag = device_tag();
    FILE *probe = fopen(path, "r");
    if (!probe) return;   // no file yet: it is created by the first append
    fclose(probe);
    // shapes fixed before the first lookup (hisq_tune_set, hisq_tune_load) stay
    if (!tag.empty()) (void)read_tune_file(path, tag, true, false, nullptr);
}

void cache_append(const TuneKey &k, const DslashTile &t, float ms) {
    const char *path = cache_path();
    if (!path) return;
    const std::string tag = device_tag();
    if (tag.empty()) return;
    FILE *fp = fopen(path, "a");
    if (!fp) return;
    const std::string l = tune_line(tag, k, t, ms);
    fputs(l.c_str(), fp);
    fclose(fp);
}

// candidate shapes for a block of c right-hand sides (c a power of two <= 16)
// grids: 0 = one tile per block; 256*k = a persistent grid of k blocks per CU
// slab_ok: the lattice is deep enough in z for the z-slab order (one plane per XCD at least)
std::vector<DslashTile> candidates(int c, bool batched_ok, bool fp32, bool slab_ok) {
    std::vector<DslashTile> v;
    const int nsweep = slab_ok ? 3 : 2;
    if (c == 1) {
        for (int st : {1, 2, 4, 8, -1, -2})
            for (int blk : {128, 256})
                for (int per_cu : {0, 4, 8})
                    for (int sw = 0; sw < nsweep; sw++)
                        v.push_back(DslashTile{1, 1, st, blk, per_cu * 256 * (256 / blk), sw});
        return v;
    }
    if (!batched_ok) return v;
    for (int nr : {1, 2, 4, 8, 16}) {
        if (nr > c) break;
        const int rg = c / nr;
        for (int grid : {0, 2048})
            for (int sw = 0; sw < nsweep; sw++) {
                v.push_back(DslashTile{nr, rg, 1, 256, grid, sw});
                if (nr == 1) v.push_back(DslashTile{nr, rg, 2, 256, grid, sw});
                // double-buffered: the next hop's words in flight during this hop's arithmetic
                if (nr > 1 && nr <= 8) v.push_back(DslashTile{nr, rg, -1, 256, grid, sw});
            }
    }
    // the matrix-core path: four lanes per site, FP32 compute only
    if (fp32 && c >= 4)
        for (int grid : {0, 2048})
            for (int sw = 0; sw < nsweep; sw++) v.push_back(DslashTile{c / 4, 4, 5, 256, grid, sw});
    return v;
}

DslashTile default_tile(int c) {
    if (c == 1) return DslashTile{1, 1, 8, 256, 0, 0};
    return DslashTile{1, c, 1, 256, 0, 0};
}

// time one shape on the probe arguments (pure Dslash, idempotent: no xpay, no reduction)
float time_tile(const DslashArgs &probe, const hisq_fmt &f, const DslashTile &t, hipStream_t st, int reps = 3) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.f;
    }
    float best = -1.f;
    int nb = 0;
    if (launch_one(probe, f, 0, t, st, &nb) == hipSuccess) {
        hipError_t e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; r++) e = launch_one(probe, f, 0, t, st, &nb);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) best = ms / reps;
    }
    (void)hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

// red: the shape for launches with a fused reduction (timed with RED_NORM into
// a scratch partial buffer: the per-RHS FP64 sums hold registers that can
// lower the occupancy of the widest shapes)
DslashTile tile_for(const hisq_fmt &f, const Geom &g, int c, const DslashArgs *probe, hipStream_t st, bool red) {
    const TuneKey key{tune_id(f, probe ? probe->long_recon : 18), g.X, g.Y, g.Z, g.T, c, red ? 1 : 0};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    cache_read_once();
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second.first;
    const bool batched_ok = has_batched_form(f);
    DslashTile best = default_tile(c);
    if (!probe || !tuning_enabled()) return best;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return best;
    DslashArgs p = *probe;
    p.x = p.y = nullptr;
    p.red = RED_NONE;
    p.guard = Guard{nullptr, 0, 0};
    p.nrhs = std::max(1, std::min(c, probe->nrhs));   // only the columns the probe's buffers hold
    // The candidates write a library-owned output, never the caller's: the
    // caller's output may alias an operand of the real launch (out == x in
    // an in-place xpay) or hold data the caller still needs.
    int cols = p.nrhs;
    if (p.cmapped) {
        cols = 1;
        for (int k = 0; k < 16; k++)
            if ((p.cvalid >> k) & 1u) cols = std::max(cols, (int)((p.cmap >> (4 * k)) & 15ull) + 1);
    }
    const size_t out_bytes = (size_t)(cols - 1) * p.field_stride + spinor_field_bytes((size_t)g.vh, f.spinor);
    char *scratch_out = nullptr;
    if (hipMalloc((void **)&scratch_out, out_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return best;
    }
    p.out = scratch_out;
    double *scratch = nullptr;
    if (red) {
        // partials of up to 16 field columns, one per block of the largest launch
        p.pstride = dslash_max_blocks(g);
        if (hipMalloc((void **)&scratch, 16 * p.pstride * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(scratch_out);
            return best;
        }
        p.red = RED_NORM;
        p.partial = scratch;
        // the fused launches are the second Dslash of a normal operator or a
        // residual, with an xpay term: time them reading one more field per
        // column (the probe's input again, read-only, the same layout)
        p.x = probe->in;
        p.a = 1.0;
    }
    // every candidate three times, then the three fastest ten times each (a
    // single noisy sample does not decide between shapes a few per cent apart)
    std::vector<std::pair<float, DslashTile>> timed;
    for (const DslashTile &t : candidates(c, batched_ok, f.compute == 32, g.Z >= 8)) {
        const float ms = time_tile(p, f, t, st);
        if (ms > 0.f) timed.emplace_back(ms, t);
    }
    std::sort(timed.begin(), timed.end(),
              [](const std::pair<float, DslashTile> &a, const std::pair<float, DslashTile> &b) { return a.first < b.first; });
    float tbest = -1.f;
    for (size_t k = 0; k < timed.size() && k < 3; k++) {
        const float ms = time_tile(p, f, timed[k].second, st, 10);
        if (ms > 0.f && (tbest < 0.f || ms < tbest)) {
            tbest = ms;
            best = timed[k].second;
        }
    }
    // The z-slab order keeps each XCD's neighbour planes in its own L2: about
    // 9 % fewer bytes fetched into L2 at nearly the same time (the other
    // orders' extra fetches hit the memory-side cache).  Within 1 % of the
    // fastest (the spread of these timings) the same shape in that order is kept.
    if (tbest > 0.f && best.sweep != 2 && g.Z >= 8) {
        DslashTile twin = best;
        twin.sweep = 2;
        const float ms = time_tile(p, f, twin, st, 10);
        if (ms > 0.f && ms <= 1.01f * tbest) {
            tbest = ms;
            best = twin;
        }
    }
    (void)hipStreamSynchronize(st);
    if (scratch) (void)hipFree(scratch);
    (void)hipFree(scratch_out);
    g_tuned[key] = std::make_pair(best, tbest);
    if (tbest > 0.f) cache_append(key, best, tbest);
    return best;
}

}  // namespace

int dslash_blocks(int n, int block) {
    int nb = (n + block - 1) / block;
    return (nb + 7) & ~7;
}

size_t dslash_max_blocks(const Geom &g) {
    return std::max((size_t)dslash_blocks(g.vh * 16, 128), (size_t)8 * g.T * slab_tiles(g, 16, 128));
}

DslashPlan dslash_plan(const hisq_fmt &f, const Geom &g, int nrhs, const DslashArgs *probe, hipStream_t st) {
    // one launch: the block of right-hand sides padded to a power of two (the
    // padding columns are masked in the kernel), so every link is read once
    DslashPlan plan;
    int c = 1;
    while (c < nrhs && c < 16) c <<= 1;
    plan.n = 1;
    plan.rhs0[0] = 0;
    plan.tile[0] = tile_for(f, g, c, probe, st, false);
    plan.tile_red[0] = c > 1 ? tile_for(f, g, c, probe, st, true) : plan.tile[0];
    return plan;
}

DslashPlan dslash_plan_lookup(const hisq_fmt &f, const Geom &g, int nrhs, int long_recon) {
    DslashPlan plan;
    int c = 1;
    while (c < nrhs && c < 16) c <<= 1;
    plan.n = 1;
    plan.rhs0[0] = 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int red = 0; red < 2; red++) {
        const TuneKey key{tune_id(f, long_recon), g.X, g.Y, g.Z, g.T, c, red};
        auto it = g_tuned.find(key);
        const DslashTile t = it != g_tuned.end() ? it->second.first : default_tile(c);
        if (red) plan.tile_red[0] = c > 1 ? t : plan.tile[0];
        else plan.tile[0] = t;
    }
    return plan;
}

hipError_t launch_dslash_multi(const MultiArgs &m, const hisq_fmt &f, int long_recon, hipStream_t st) {
    switch (triplet_key(f)) {
    case GF_F64 * 100 + SF_F64 * 10 + 1: return dslash_multi_double(m, long_recon, st);
    case GF_F32 * 100 + SF_F32 * 10 + 0: return dslash_multi_single(m, long_recon, st);
    case GF_FIX16 * 100 + SF_HALF16 * 10 + 0: return dslash_multi_half(m, long_recon, st);
    case GF_FIX16 * 100 + SF_INT20 * 10 + 0: return dslash_multi_int20(m, long_recon, st);
    case GF_FIX32 * 100 + SF_INT30 * 10 + 1: return dslash_multi_int30(m, long_recon, st);
    case GF_FIX32 * 100 + SF_INT30 * 10 + 0: return dslash_multi_int30_fp32(m, long_recon, st);
    case GF_FIX32 * 100 + SF_INT24 * 10 + 0: return dslash_multi_int24(m, long_recon, st);
    case GF_SX24 * 100 + SF_INT24 * 10 + 0: return dslash_multi_sx24(m, long_recon, st);
    case GF_SX24 * 100 + SF_INT30 * 10 + 1: return dslash_multi_sx24_int30(m, long_recon, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dslash(const DslashArgs &a, const hisq_fmt &f, const DslashPlan &plan, hipStream_t st, int *nblocks) {
    for (int i = 0; i < plan.n; i++) {
        int nb = 0;
        const DslashTile &t = a.red != RED_NONE ? plan.tile_red[i] : plan.tile[i];
        hipError_t e = launch_one(a, f, plan.rhs0[i], t, st, &nb);
        if (e != hipSuccess) return e;
        if (nblocks)
            for (int j = 0; j < t.nr * t.rg; j++) nblocks[plan.rhs0[i] + j] = nb;
    }
    return hipSuccess;
}

}  // namespace hisq

namespace hisq {
namespace {
// fused: 0 = the plain and the fused-reduction shape, 1 = the fused-reduction shape only
hisq_status tune_set_impl(const char *who, hisq_fmt fmt, const int dims[4], int long_recon, int rhs_block, int nr,
                          int rg, int stage, int block, int grid, int sweep, int fused) {
    if (!dims || !dims_ok(dims) || !triplet_ok(fmt)) return set_error(HISQ_EINVAL, "%s: bad dims or triplet", who);
    if (long_recon != HISQ_RECON_18 && long_recon != HISQ_RECON_12 && long_recon != HISQ_RECON_8)
        return set_error(HISQ_EINVAL, "%s: long_recon must be 18, 12 or 8", who);
    const bool pow2 = rhs_block >= 1 && rhs_block <= 16 && (rhs_block & (rhs_block - 1)) == 0;
    if (!pow2) return set_error(HISQ_EINVAL, "%s: rhs_block must be 1, 2, 4, 8 or 16", who);
    if (fused && rhs_block == 1)
        return set_error(HISQ_EINVAL, "%s: one right-hand side has a single shape (use hisq_tune_set)", who);
    if (rhs_block > 1 && !has_batched_form(fmt)) return set_error(HISQ_EINVAL, "%s: this triplet has no batched Dslash", who);
    if (!recon_ok(fmt, long_recon, rhs_block > 1))
        return set_error(HISQ_EINVAL, "%s: eight-parameter long links: FP64 triplets with F64 or FIX32 links, one "
                                      "right-hand side", who);
    if (!shape_ok(fmt, rhs_block, DslashTile{nr, rg, stage, block, grid, sweep}))
        return set_error(HISQ_EINVAL, "%s: unsupported shape nr %d rg %d stage %d block %d grid %d sweep %d", who, nr,
                         rg, stage, block, grid, sweep);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (int red = fused ? 1 : 0; red < (rhs_block > 1 ? 2 : 1); red++) {
        const TuneKey key{tune_id(fmt, long_recon), dims[0], dims[1], dims[2], dims[3], rhs_block, red};
        g_tuned[key] = std::make_pair(DslashTile{nr, rg, stage, block, grid, sweep}, -1.f);
    }
    return HISQ_OK;
}
}  // namespace
}  // namespace hisq

extern "C" hisq_status hisq_tune_set(hisq_fmt fmt, const int dims[4], int long_recon, int rhs_block, int nr, int rg,
                                     int stage, int block, int grid, int sweep) {
    return hisq::tune_set_impl("hisq_tune_set", fmt, dims, long_recon, rhs_block, nr, rg, stage, block, grid, sweep, 0);
}

extern "C" hisq_status hisq_tune_set_fused(hisq_fmt fmt, const int dims[4], int long_recon, int rhs_block, int nr,
                                           int rg, int stage, int block, int grid, int sweep) {
    return hisq::tune_set_impl("hisq_tune_set_fused", fmt, dims, long_recon, rhs_block, nr, rg, stage, block, grid,
                               sweep, 1);
}

extern "C" void hisq_tune_clear(void) {
    std::lock_guard<std::mutex> lk(hisq::g_tune_mu);
    hisq::g_tuned.clear();
    hisq::g_cache_read = true;   // a cleared table is not refilled from HISQ_TUNE_CACHE
}

extern "C" hisq_status hisq_tune_save(const char *path) {
    if (!path) return hisq::set_error(HISQ_EINVAL, "hisq_tune_save: null path");
    const std::string tag = hisq::device_tag();
    if (tag.empty()) return hisq::set_error(HISQ_EHIP, "hisq_tune_save: no current HIP device");
    std::string body = "# libhisq launch shapes (hisq_tune_save)\n";
    {
        std::lock_guard<std::mutex> lk(hisq::g_tune_mu);
        for (const auto &kv : hisq::g_tuned) body += hisq::tune_line(tag, kv.first, kv.second.first, kv.second.second);
    }
    const std::string tmp = std::string(path) + ".tmp";
    FILE *fp = fopen(tmp.c_str(), "w");
    if (!fp) return hisq::set_error(HISQ_EIO, "hisq_tune_save: cannot write %s", tmp.c_str());
    const bool ok = fwrite(body.data(), 1, body.size(), fp) == body.size();
    if (fclose(fp) != 0 || !ok || rename(tmp.c_str(), path) != 0) {
        (void)remove(tmp.c_str());
        return hisq::set_error(HISQ_EIO, "hisq_tune_save: cannot write %s", path);
    }
    return HISQ_OK;
}

extern "C" hisq_status hisq_tune_load(const char *path, int *nloaded) {
    if (nloaded) *nloaded = 0;
    if (!path) return hisq::set_error(HISQ_EINVAL, "hisq_tune_load: null path");
    const std::string tag = hisq::device_tag();
    if (tag.empty()) return hisq::set_error(HISQ_EHIP, "hisq_tune_load: no current HIP device");
    std::lock_guard<std::mutex> lk(hisq::g_tune_mu);
    return hisq::read_tune_file(path, tag, true, true, nloaded);
}

extern "C" size_t hisq_tune_report(char *buf, size_t len) {
    std::string s;
    {
        std::lock_guard<std::mutex> lk(hisq::g_tune_mu);
        for (const auto &kv : hisq::g_tuned) {
            char line[256];
            const auto &k = kv.first;
            const auto &t = kv.second.first;
            snprintf(line, sizeof(line),
                     "triplet %03d recon %d lattice %dx%dx%dx%d rhs-block %d%s: nr %d rg %d stage %d block %d grid %d "
                     "sweep %d (%.1f us)\n",
                     std::get<0>(k) / 100, std::get<0>(k) % 100, std::get<1>(k), std::get<2>(k), std::get<3>(k),
                     std::get<4>(k), std::get<5>(k), std::get<6>(k) ? " reduction" : "",
                     t.nr, t.rg, t.stage, t.block, t.grid, t.sweep, kv.second.second * 1e3);
            s += line;
        }
    }
    if (buf && len) {
        const size_t n = s.size() < len - 1 ? s.size() : len - 1;
        memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return s.size() + 1;
}
