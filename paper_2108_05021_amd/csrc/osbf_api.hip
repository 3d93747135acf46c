// C ABI of the one-sided box filter: argument validation, launch planning and
// the sweep driver.  All device work is enqueued on the caller's stream.
#include <iterator>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../../include/osbf.h"
#include "osbf_internal.h"

using namespace osbf;

namespace {

thread_local std::string g_last_error;

osbf_status fail(osbf_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
osbf_status fail(osbf_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

osbf_status hip_fail(hipError_t e, const char *what) {
    return fail(OSBF_ERROR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t elem_bytes(osbf_dtype dt) { return dt == OSBF_F32 ? 4 : 2; }

bool valid_dtype(int dt) { return dt == OSBF_F32 || dt == OSBF_F16 || dt == OSBF_BF16; }

// Largest dynamic LDS a workgroup may use on the current device.
size_t lds_limit() {
    static std::mutex mu;
    static std::vector<size_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (!cache[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess || v <= 0)
            if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
                v = 65536;
        cache[dev] = (size_t)v;
    }
    return cache[dev];
}

struct Plan {
    int geom = GEOM_GENERIC;
    int tw = 0, th = 0;  // output tile (multiples of r); tw == 0: nothing fits
    int k = 1;           // sweeps fused per launch
    int pitch = 0, arr = 0;
    size_t lds = 0;      // streaming kernel: its LDS bytes (th: rows per workgroup)
    size_t lds_bytes() const { return lds ? lds : (size_t)4 * arr * sizeof(float); }
};

// LDS regions (width x height, halo included) the generic kernel considers.
const int kRegions[][2] = {{64, 64}, {128, 64}, {64, 128}, {96, 96}, {128, 128}, {256, 64},
                           {64, 32}, {32, 32}, {80, 80}, {104, 96}};

Plan make_plan(int geom, int RW, int RH, int r, int k) {
    Plan p;
    if (stream_geom(geom)) {  // one or two sweeps per launch; strips of whole blocks of r columns
        if (!fixed_radius(r) || k > 2 || (k == 2 && !stream_fusable(RW, r))) return Plan{};
        const int tw = ((RW - 2 * k * r) / r) * r;
        if (tw < std::max(r, 4)) return Plan{};
        p.geom = geom;
        p.tw = tw;
        p.th = 0;  // rows per workgroup chosen at launch to fill the device once
        p.k = k;
        p.lds = k == 2 ? stream2_lds_bytes(RW, r) : stream_lds_bytes(RW, r);
        return p;
    }
    if (!fwd_tile_shape(RW, RH, r, k, &p.tw, &p.th)) return Plan{};
    p.geom = geom;
    p.k = k;
    if (geom == GEOM_GENERIC) {
        fwd_lds_layout(p.tw, p.th, r, k, &p.pitch, &p.arr);
    } else {
        p.pitch = RW + 1;
        p.arr = RH * p.pitch;
    }
    return p;
}

// Cost per output pixel-sweep: selection work over the fused sweeps' grown
// regions (halo recomputation), the cheaper running-sum phases and the halo
// load, HBM traffic that shrinks as 1/k, and a penalty for low occupancy.
double plan_cost(const Plan &p, int H, int W, int r) {
    if (stream_geom(p.geom))  // selection on tw of RW columns, no vertical halo to speak of
        return 0.75 * kGeomDims[p.geom][0] / std::min(p.tw, W) + 0.25 / p.k;
    const double tw = std::min(p.tw, W), th = std::min(p.th, H);
    double work = 0;
    for (int j = 0; j < p.k; ++j) {
        const double e = (double)(p.k - 1 - j) * r;
        const double cw = std::min<double>(tw + 2 * e, W), ch = std::min<double>(th + 2 * e, H);
        work += cw * ch * 1.0 + (cw + 2 * r) * (ch + r) * 0.08 + (cw + r) * (ch + r) * 0.15;
    }
    const double lw = std::min<double>(tw + 2.0 * p.k * r, W), lh = std::min<double>(th + 2.0 * p.k * r, H);
    work += lw * lh * 0.05;
    double cost = work / ((double)p.k * tw * th);
    // waves resident per CU: LDS-limited workgroups times waves per workgroup
    const int per_cu = (int)(163840 / std::max<size_t>(p.lds_bytes(), 1));
    const int waves = per_cu * (p.geom == GEOM_GENERIC ? 4 : (p.geom == GEOM_128x64 ? 16 : 8));
    if (waves < 8) cost *= 1.8;
    else if (waves < 12) cost *= 1.3;
    else if (waves < 16) cost *= 1.1;
    if (p.geom == GEOM_GENERIC) cost *= 1.8;   // runtime-pitch addressing
    return cost + 0.25 / p.k;
}

// Measured defaults for the compiled radii (3x2048x2048 FP32, T=30 on
// MI355X, plan sweep over geometries, fusion depths, streaming strip widths
// and rows per workgroup, 0 = chosen to fill the device once), in order of
// preference: the row-streaming kernel, one sweep per launch, except at
// r = 1, where the fused two-sweep kernel is 6-10% faster (20.4-21.1 against
// 21.6-23.4 us per sweep; at r = 2 it is 5% slower, at r = 3 even); the
// later entries are fallbacks for devices whose LDS does not fit the first.
// At r = 4, 8 and 16 the 128-lane strips have the smallest worst-case ratio
// to the fastest plan over 3x2048^2, 1x4096^2, 2x2000x3000, 8x1024^2 and
// 1x1400^2 (T=10: 1.04, 1.03, 1.05 against 1.07, 1.07, 1.05 for 192-lane
// strips, which are at most 1.3% faster on 3x2048^2).  At r = 2, 5 and 10
// the plans are the fastest on 3x2048^2; on other shapes 192-lane strips at
// r = 5 gain up to 10% and the fused 128-lane kernel at r = 2 up to 5%,
// which the autotuner finds.
struct TunedShape { int r, geom, k, rows; };
const TunedShape kTuned[] = {{1, GEOM_S128, 2, 0}, {1, GEOM_64x48, 3, 0},
                             {2, GEOM_S192, 1, 0}, {2, GEOM_64x48, 2, 0},
                             {3, GEOM_S128, 1, 0}, {3, GEOM_64x48, 2, 0},
                             {4, GEOM_S128, 1, 0}, {4, GEOM_64x48, 1, 0},
                             {5, GEOM_S128, 1, 0}, {5, GEOM_64x60, 1, 0},
                             {8, GEOM_S128, 1, 0}, {8, GEOM_64x48, 1, 0},
                             {10, GEOM_S192, 1, 0}, {10, GEOM_64x60, 1, 0},
                             {16, GEOM_S128, 1, 0}, {16, GEOM_128x64, 1, 0}};

// From 2^20 up to 2^21 plane-pixels at r = 1 and 2 the tiled kernel with
// fused sweeps still beats the streaming plans (1x1024^2 / 1x1400^2, T=10,
// us per sweep: r=1 4.43 / 6.70 against 5.43 / 7.02, r=2 4.99 / 7.68
// against 7.25 / 9.01); from r = 3 up the streaming plans are within 1.19x
// of the best there.
const TunedShape kTunedMid[] = {{1, GEOM_64x60, 5, 0}, {2, GEOM_64x48, 2, 0}};

// Images below 2^20 plane-pixels are launch- and latency-bound: a few short
// launches of the tiled kernel with several fused sweeps beat the streaming
// kernel, whose few workgroups then run long serial chains of steps.  Two
// tables, measured on MI355X at T=10, FP32: below 2^17 plane-pixels (1x64^2,
// 1x128x160, 1x256^2) and from 2^17 to 2^20 (3x300x400, 1x700x900,
// 3x512^2); each entry is the plan with the smallest worst-case ratio to each
// shape's fastest (within 1.0-1.15x of it below 2^17 and 1.05-1.24x above,
// where one table for both ranges was up to 1.42x slower and the large-image
// table up to 4.6x).
const TunedShape kTunedTiny[] = {{1, GEOM_64x32, 8, 0}, {2, GEOM_64x32, 6, 0}, {3, GEOM_64x48, 6, 0},
                                 {4, GEOM_64x48, 4, 0}, {5, GEOM_64x60, 4, 0}, {8, GEOM_64x48, 2, 0},
                                 {10, GEOM_64x60, 2, 0}, {16, GEOM_64x60, 1, 0}};
const TunedShape kTunedSmall[] = {{1, GEOM_64x48, 6, 0}, {2, GEOM_64x60, 5, 0}, {3, GEOM_64x60, 3, 0},
                                  {4, GEOM_64x60, 2, 0}, {5, GEOM_64x60, 2, 0}, {8, GEOM_64x60, 1, 0},
                                  {10, GEOM_64x60, 1, 0}, {16, GEOM_128x64, 1, 0}};

// Above 2^25 plane-pixels, two more tables.  While the ping-pong (two
// iterates) is larger than the 256 MiB Infinity Cache (FP32, or 16-bit
// storage above 2^26 pixels), every sweep reads and writes DRAM: two fused
// sweeps per launch (half the DRAM bytes per sweep) then pay from r = 1 to 4,
// 256-lane strips with 64-row chunks at r = 5 and 128-lane strips at r = 16
// (measured on 1x8192^2 and 3x4096^2, FP32, T=10, best of two passes in
// opposite orders, us per sweep against the large-image table's plan: r=1
// 91.0 / 71.0 (96.1 / 72.3), r=2 101.0 / 78.5 (128.3 / 93.1), r=3 102.8 /
// 78.5 (127.0 / 95.4), r=4 111.7 / 87.3 (135.9 / 100.9), r=5 118.4 / 92.0
// (159.9 / 113.9), r=16 178.1 / 140.9 (186.0 / 147.3); r=8 and 10 keep
// theirs).  16-bit storage up to 2^26 pixels (a ping-pong within the cache)
// takes one sweep per launch with 64-row chunks, which there beat both the
// fused plans and the chunks that fill the device once (1x8192^2 BF16 and
// FP16: r=2 87.3 against 93.0 and 103.0 us, r=4 92.7 against 112.7 and
// 116.1, r=5 100.2 against 129.7).
const TunedShape kTunedDram[] = {{1, GEOM_S128, 2, 64}, {1, GEOM_64x48, 3, 0},
                                 {2, GEOM_S192, 2, 64}, {2, GEOM_64x48, 2, 0},
                                 {3, GEOM_S192, 2, 0}, {3, GEOM_64x48, 2, 0},
                                 {4, GEOM_S192, 2, 0}, {4, GEOM_64x48, 1, 0},
                                 {5, GEOM_S256, 1, 64}, {5, GEOM_64x60, 1, 0},
                                 {8, GEOM_S192, 1, 0}, {8, GEOM_64x48, 1, 0},
                                 {10, GEOM_S192, 1, 0}, {10, GEOM_64x60, 1, 0},
                                 {16, GEOM_S128, 1, 0}, {16, GEOM_128x64, 1, 0}};
const TunedShape kTunedHuge[] = {{1, GEOM_S128, 1, 0}, {1, GEOM_64x48, 3, 0},
                                 {2, GEOM_S128, 1, 64}, {2, GEOM_64x48, 2, 0},
                                 {3, GEOM_S128, 1, 64}, {3, GEOM_64x48, 2, 0},
                                 {4, GEOM_S128, 1, 64}, {4, GEOM_64x48, 1, 0},
                                 {5, GEOM_S256, 1, 64}, {5, GEOM_64x60, 1, 0},
                                 {8, GEOM_S192, 1, 0}, {8, GEOM_64x48, 1, 0},
                                 {10, GEOM_S192, 1, 0}, {10, GEOM_64x60, 1, 0},
                                 {16, GEOM_S128, 1, 0}, {16, GEOM_128x64, 1, 0}};

// Autotune cache: (device model, radius, dtype, size class) -> plan measured
// by osbf_autotune, and (device model, dtype, radius) -> rows per batched
// work item measured by osbf_batched_autotune.  Guarded by a mutex; every
// plan gives the same bits, so the cache changes speed only.  With
// OSBF_TUNE_CACHE naming a file, the cache is read from it on first use and
// written back after every tuning call (device models are keyed by their
// architecture name and CU count, so a file carries over between processes
// and machines of one model).
std::mutex g_tune_mu;
std::map<std::tuple<std::string, int, int, int>, Plan> g_tune;
std::map<std::tuple<std::string, int, int>, int> g_tune_batch;
bool g_tune_file_read = false;

// "<gcnArchName>:<CUs>" of a device ("" on error); cached per device index.
std::string device_model(int dev) {
    static std::mutex mu;
    static std::map<int, std::string> names;
    std::lock_guard<std::mutex> lock(mu);
    auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
    std::string name = prop.gcnArchName;
    for (char &c : name)
        if (c == ' ') c = '_';
    name += ":" + std::to_string(prop.multiProcessorCount);
    names[dev] = name;
    return name;
}

std::string current_model() {
    int dev = 0;
    return hipGetDevice(&dev) == hipSuccess ? device_model(dev) : std::string();
}

// A cached plan from its stored fields (geometry, fusion depth, region of
// the generic kernel, rows of the streaming kernel); tw == 0 if malformed.
Plan plan_from_fields(int geom, int rw, int rh, int k, int th, int r) {
    if (geom < 0 || geom >= NUM_GEOMS || k < 1 || k > 8 || r < 1 || r > OSBF_MAX_RADIUS || th < 0) return Plan{};
    if (geom != GEOM_GENERIC) rw = kGeomDims[geom][0], rh = kGeomDims[geom][1];
    if (rw <= 0 || rw > 1024 || rh < 0 || rh > 1024) return Plan{};
    Plan p = make_plan(geom, rw, rh, r, k);
    if (stream_geom(geom)) p.th = th;
    return p;
}

// Region of a generic plan (the LDS region its tile came from), for storing.
void plan_region(const Plan &p, int r, int *rw, int *rh) {
    *rw = kGeomDims[p.geom][0];
    *rh = kGeomDims[p.geom][1];
    if (p.geom == GEOM_GENERIC) {
        *rw = p.tw + 2 * p.k * r;
        *rh = p.th + 2 * p.k * r;
    }
}

// Caller holds g_tune_mu.
void tune_file_read_locked() {
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char *path = getenv("OSBF_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[512], model[256];
    while (fgets(line, sizeof line, f)) {
        int r, dt, cls, geom, rw, rh, k, th, rows;
        if (sscanf(line, "fwd %255s %d %d %d %d %d %d %d %d", model, &r, &dt, &cls, &geom, &rw, &rh, &k, &th) == 9) {
            const Plan p = plan_from_fields(geom, rw, rh, k, th, r);
            if (p.tw && valid_dtype(dt) && cls >= 0 && cls <= 3)
                g_tune[std::make_tuple(std::string(model), r, dt, cls)] = p;
        } else if (sscanf(line, "batch %255s %d %d %d", model, &dt, &r, &rows) == 4) {
            if (valid_dtype(dt) && r >= 1 && r <= OSBF_MAX_RADIUS && rows >= 1 && rows <= 4096)
                g_tune_batch[std::make_tuple(std::string(model), dt, r)] = rows;
        }
    }
    fclose(f);
}

// Caller holds g_tune_mu.  Writes the whole cache (tmp file, then rename).
void tune_file_write_locked() {
    const char *path = getenv("OSBF_TUNE_CACHE");
    if (!path || !*path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "# osbf autotune cache: fwd model r dtype class geom region_w region_h k rows | "
               "batch model dtype r rows\n");
    for (const auto &kv : g_tune) {
        const Plan &p = kv.second;
        int rw, rh;
        plan_region(p, std::get<1>(kv.first), &rw, &rh);
        fprintf(f, "fwd %s %d %d %d %d %d %d %d %d\n", std::get<0>(kv.first).c_str(), std::get<1>(kv.first),
                std::get<2>(kv.first), std::get<3>(kv.first), p.geom, rw, rh, p.k, std::max(p.th, 0));
    }
    for (const auto &kv : g_tune_batch)
        fprintf(f, "batch %s %d %d %d\n", std::get<0>(kv.first).c_str(), std::get<1>(kv.first),
                std::get<2>(kv.first), kv.second);
    const bool ok = fclose(f) == 0;
    if (ok) rename(tmp.c_str(), path);
}

// 0: below 2^17 plane-pixels, 1: below 2^20, 2: up to 2^25, 3: larger.
int size_class(int planes, int H, int W) {
    const long long px = (long long)planes * H * W;
    return px < (1LL << 17) ? 0 : px < (1LL << 20) ? 1 : px <= (1LL << 25) ? 2 : 3;
}

// Rows per workgroup of a plan (the streaming kernel rounds to whole steps;
// 0: chosen at launch so that the chunks fill the device's resident
// workgroup slots once).
int plan_rows(const Plan &p, int r) {
    if (!stream_geom(p.geom) || p.th <= 0) return p.th;
    const int step = stream_step(r);
    return (p.th + step - 1) / step * step;
}

bool tuned_plan(int planes, int H, int W, int r, int T, int dtype, Plan *out) {
    const std::string model = current_model();
    if (model.empty()) return false;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_file_read_locked();
    auto it = g_tune.find(std::make_tuple(model, r, dtype, size_class(planes, H, W)));
    if (it == g_tune.end()) return false;
    const Plan &p = it->second;
    if (p.k > std::min(T, 8)) return false;  // fewer sweeps than the tuned fusion
    if (stream_geom(p.geom) && !stream_width_ok(W, 4, r, std::max(p.th, stream_step(r)))) return false;
    *out = p;
    return true;
}

Plan choose_plan_model(int planes, int H, int W, int r, int T, int dtype);

// The launch plan: OSBF_PLAN if set, else an autotuned plan for this device
// and problem class, else the measured table of the problem's size class,
// else the cost model.
Plan choose_plan(int planes, int H, int W, int r, int T, int dtype) {
    Plan p;
    if (!getenv("OSBF_PLAN") && tuned_plan(planes, H, W, r, T, dtype, &p)) return p;
    return choose_plan_model(planes, H, W, r, T, dtype);
}

// OSBF_PLAN="geom,k[,rows]" forces a plan (tests and tuning): geom 0 is the
// generic kernel (region chosen by cost), 1.. the fixed and streaming
// geometries (enum Geom); rows sets the streaming kernel's rows per workgroup.
Plan choose_plan_model(int planes, int H, int W, int r, int T, int dtype) {
    const size_t limit = lds_limit();
    const int kmax = T > 0 ? std::min(T, 8) : 1;
    int force_geom = -1, force_k = -1, force_rows = 0;
    if (const char *env = getenv("OSBF_PLAN")) {
        const int n = sscanf(env, "%d,%d,%d", &force_geom, &force_k, &force_rows);
        if (n < 2 || force_geom < 0 || force_geom >= NUM_GEOMS || force_k < 1 || force_rows < 0)
            force_geom = force_k = -1, force_rows = 0;
        else
            force_k = std::min(force_k, kmax);
    }
    if (force_geom < 0) {
        const int cls = size_class(planes, H, W);
        if (cls < 2) {
            for (const auto &t : cls == 0 ? kTunedTiny : kTunedSmall) {
                if (t.r != r) continue;
                Plan p = make_plan(t.geom, kGeomDims[t.geom][0], kGeomDims[t.geom][1], r, std::min(t.k, kmax));
                if (p.tw && p.lds_bytes() <= limit) return p;
            }
        }
        if (cls == 2 && (long long)planes * H * W < (1LL << 21)) {
            for (const auto &t : kTunedMid) {
                if (t.r != r) continue;
                Plan p = make_plan(t.geom, kGeomDims[t.geom][0], kGeomDims[t.geom][1], r, std::min(t.k, kmax));
                if (p.tw && p.lds_bytes() <= limit) return p;
            }
        }
        // above 2^25 pixels: DRAM-bound while the two iterates outgrow the
        // 256 MiB Infinity Cache
        const bool dram = (long long)planes * H * W * (long long)elem_bytes((osbf_dtype)dtype) * 2 > (256LL << 20);
        const TunedShape *tab = cls < 3 ? kTuned : dram ? kTunedDram : kTunedHuge;
        const size_t ntab = cls < 3 ? std::size(kTuned) : dram ? std::size(kTunedDram) : std::size(kTunedHuge);
        for (size_t i = 0; i < ntab; ++i) {
            const TunedShape &t = tab[i];
            if (t.r != r) continue;
            if (stream_geom(t.geom) && !stream_width_ok(W, 4, r, stream_step(r))) continue;
            Plan p = make_plan(t.geom, kGeomDims[t.geom][0], kGeomDims[t.geom][1], r, std::min(t.k, kmax));
            if (stream_geom(t.geom)) p.th = t.rows;
            if (p.tw && p.lds_bytes() <= limit) return p;
        }
    }
    Plan best;
    double best_cost = 1e300;
    auto consider = [&](const Plan &p) {
        if (!p.tw || p.lds_bytes() > limit) return;
        if (stream_geom(p.geom) && !stream_width_ok(W, 4, r, stream_step(r))) return;
        const double c = plan_cost(p, H, W, r);
        if (c < best_cost) { best_cost = c; best = p; }
    };
    for (int k = 1; k <= kmax; ++k) {
        if (force_k > 0 && k != force_k) continue;
        if (fixed_radius(r))
            for (int g = 1; g < NUM_GEOMS; ++g)
                if (force_geom < 0 || force_geom == g)
                    consider(make_plan(g, kGeomDims[g][0], kGeomDims[g][1], r, k));
        if (force_geom <= 0)
            for (const auto &reg : kRegions) consider(make_plan(GEOM_GENERIC, reg[0], reg[1], r, k));
    }
    if (best.tw && stream_geom(best.geom) && force_rows > 0) best.th = force_rows;
    if (!best.tw && force_geom >= 0) {   // forced plan does not fit: fall back to the model
        for (int k = 1; k <= kmax; ++k) {
            if (fixed_radius(r))
                for (int g = 1; g < NUM_GEOMS; ++g) consider(make_plan(g, kGeomDims[g][0], kGeomDims[g][1], r, k));
            for (const auto &reg : kRegions) consider(make_plan(GEOM_GENERIC, reg[0], reg[1], r, k));
        }
    }
    return best;
}

struct Launch {
    int t0, k;  // first sweep, sweeps in this launch
};

// Segments of ck sweeps (when checkpointing), each cut into launches of at
// most k sweeps; recomputing one segment replays exactly the same launches.
std::vector<Launch> make_launches(int T, int ck, int k) {
    std::vector<Launch> v;
    const int seg = ck > 0 ? ck : T;
    for (int s0 = 0; s0 < T; s0 += seg) {
        const int s1 = std::min(T, s0 + seg);
        for (int t = s0; t < s1; t += k) v.push_back(Launch{t, std::min(k, s1 - t)});
    }
    return v;
}

// Enqueue one forward launch (k sweeps from t0) over every plane, chunked so
// the grid stays within 2^31 workgroups.  `sel_t0` is the map of sweep t0,
// plane 0 (nullable); consecutive sweeps' maps are plane_set apart.
hipError_t enqueue_forward(const Plan &plan, int k, const void *in, void *out, uint8_t *sel_t0,
                           int planes, int H, int W, int r, osbf_dtype dtype, hipStream_t stream,
                           int mode = 0) {
    const size_t plane_set = (size_t)planes * H * W;
    const int th = plan_rows(plan, r);
    const int tiles_x = (W + plan.tw - 1) / plan.tw, tiles_y = th > 0 ? (H + th - 1) / th : 1;
    const int max_planes = std::max(1, (int)(((1LL << 31) - 1) / ((long long)tiles_x * tiles_y)));
    for (int p0 = 0; p0 < planes; p0 += max_planes) {
        const int np = std::min(max_planes, planes - p0);
        const size_t off = (size_t)p0 * H * W;
        FwdLaunch a;
        a.src = (const char *)in + off * elem_bytes(dtype);
        a.dst = (char *)out + off * elem_bytes(dtype);
        a.sel = sel_t0 ? sel_t0 + off : nullptr;
        a.sel_stride = (long long)plane_set;
        a.planes = np;
        a.H = H; a.W = W; a.r = r; a.k = k;
        a.tw = plan.tw; a.th = th;
        a.tiles_x = tiles_x; a.tiles_y = tiles_y;
        a.geom = plan.geom;
        if (plan.geom == GEOM_GENERIC)
            fwd_lds_layout(plan.tw, plan.th, r, k, &a.pitch, &a.arr);
        else
            a.pitch = plan.pitch, a.arr = plan.arr;
        hipError_t e = mode ? launch_forward_mode(mode, (int)dtype, a, stream) : launch_forward((int)dtype, a, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Adjoint kernel choice: the row-streaming kernel for its radii, then the
// fixed-geometry tiled kernel, then the smallest square region of the generic
// kernel that fits the device's LDS.  OSBF_ADJOINT=fixed or generic forces
// the tiled kernels (tests compare all of them bit for bit);
// OSBF_ADJOINT_ROWS sets the streaming kernel's rows per workgroup (rounded
// up to whole blocks of r; tests and tuning).
bool adjoint_tile(int r, int W, BwdLaunch *b) {
    const char *env = getenv("OSBF_ADJOINT");
    const bool force_generic = env && strcmp(env, "generic") == 0;
    const bool force_fixed = env && strcmp(env, "fixed") == 0;
    b->fixed = 0;
    size_t fixed_lds = 0;
    const bool stream = !force_generic && !force_fixed && adjoint_stream_tile(r, &b->tw, &b->th, &fixed_lds);
    if (stream) {
        const char *rows = getenv("OSBF_ADJOINT_ROWS");
        const int n = rows ? atoi(rows) : 0;
        if (n > 0 && n <= 4096) b->th = (n + r - 1) / r * r;
    }
    // (the streaming kernel addresses a chunk's rows through 32-bit offsets)
    if (stream &&
        fixed_lds <= lds_limit() && (long long)(b->th + 6 * r) * W * 4 < (1LL << 31)) {
        b->fixed = 2;
        b->pitch = b->arr = 0;
        return true;
    }
    if (!force_generic && adjoint_fixed_tile(r, &b->tw, &b->th, &fixed_lds) && fixed_lds <= lds_limit()) {
        b->fixed = 1;
        b->pitch = b->arr = 0;
        return true;
    }
    for (int reg : {64, 80, 96, 128}) {
        const int t = ((reg - 4 * r) / r) * r;
        if (t < std::max(r, 4)) continue;
        bwd_lds_layout(t, t, r, &b->pitch, &b->arr);
        if ((size_t)5 * b->arr * sizeof(float) <= lds_limit()) {
            b->tw = b->th = t;
            return true;
        }
    }
    return false;
}

osbf_status check_sizes(int32_t planes, int32_t H, int32_t W, int dtype, int32_t r, int32_t T) {
    if (planes < 1 || H < 1 || W < 1)
        return fail(OSBF_ERROR_INVALID_VALUE, "planes, height and width must be >= 1 (got %d, %d, %d)",
                    planes, H, W);
    if ((long long)H * W > (1LL << 40))
        return fail(OSBF_ERROR_INVALID_VALUE, "plane too large");
    if (!valid_dtype(dtype)) return fail(OSBF_ERROR_INVALID_VALUE, "unknown dtype %d", dtype);
    if (r < 0 || r > OSBF_MAX_RADIUS)
        return fail(OSBF_ERROR_INVALID_VALUE, "radius %d outside [0, %d]", r, OSBF_MAX_RADIUS);
    if (T < 0) return fail(OSBF_ERROR_INVALID_VALUE, "iterations %d < 0", T);
    return OSBF_SUCCESS;
}

}  // namespace

extern "C" {

int32_t osbf_abi_version(void) { return OSBF_ABI_VERSION; }

const char *osbf_status_string(osbf_status s) {
    switch (s) {
    case OSBF_SUCCESS: return "success";
    case OSBF_ERROR_INVALID_VALUE: return "invalid value";
    case OSBF_ERROR_UNSUPPORTED: return "unsupported";
    case OSBF_ERROR_WORKSPACE: return "workspace missing or too small";
    case OSBF_ERROR_HIP: return "HIP runtime error";
    case OSBF_ERROR_TIMEOUT: return "device wait timed out";
    }
    return "unknown status";
}

const char *osbf_last_error(void) { return g_last_error.c_str(); }

size_t osbf_forward_workspace_size(int32_t planes, int32_t H, int32_t W, osbf_dtype dtype,
                                   int32_t r, int32_t T) {
    if (check_sizes(planes, H, W, dtype, r, T) != OSBF_SUCCESS) return (size_t)-1;
    if (T == 0 || r == 0) return 0;
    return (size_t)planes * H * W * elem_bytes(dtype);
}

}  // extern "C"

namespace {
osbf_status forward_impl(const void *src, void *dst, int32_t planes, int32_t H, int32_t W,
                         osbf_dtype dtype, int32_t r, int32_t T, osbf_boundary boundary,
                         uint8_t *sel, void *ckpt, int32_t ck, void *ws, size_t ws_bytes,
                         void *stream_, int mode) {
    g_last_error.clear();
    osbf_status st = check_sizes(planes, H, W, dtype, r, T);
    if (st != OSBF_SUCCESS) return st;
    if (boundary != OSBF_BOUNDARY_REPLICATE)
        return fail(OSBF_ERROR_INVALID_VALUE, "unknown boundary %d", (int)boundary);
    if (!src || !dst) return fail(OSBF_ERROR_INVALID_VALUE, "src and dst must be non-NULL");
    if (ckpt && ck < 1) return fail(OSBF_ERROR_INVALID_VALUE, "checkpoint interval %d < 1", ck);
    hipStream_t stream = (hipStream_t)stream_;
    const size_t plane_set = (size_t)planes * H * W;
    const size_t bytes = plane_set * elem_bytes(dtype);
    const int nck = (ckpt && T > 0) ? (T + ck - 1) / ck : 0;
    hipError_t e;

    if (T == 0 || r == 0) {  // identity; every window is the pixel itself when r = 0
        if (src != dst && (e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
            return hip_fail(e, "copy");
        if (sel && T > 0 && (e = hipMemsetAsync(sel, OSBF_WIN_R, (size_t)T * plane_set, stream)) != hipSuccess)
            return hip_fail(e, "memset sel");
        for (int s = 0; s < nck; ++s)
            if ((e = hipMemcpyAsync((char *)ckpt + s * bytes, src, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
                return hip_fail(e, "copy checkpoint");
        return OSBF_SUCCESS;
    }

    const Plan plan = choose_plan(planes, H, W, r, T, (int)dtype);
    if (!plan.tw)
        return fail(OSBF_ERROR_UNSUPPORTED, "radius %d does not fit the device's LDS", r);
    const std::vector<Launch> launches = make_launches(T, nck ? ck : 0, plan.k);
    const int nl = (int)launches.size();
    const bool need_ws = nl >= 2 || src == dst;
    if (need_ws && (!ws || ws_bytes < bytes))
        return fail(OSBF_ERROR_WORKSPACE, "workspace of %zu bytes required, got %zu", bytes, ws ? ws_bytes : 0);

    const void *cur = src;
    if (src == dst && (nl % 2) == 1) {
        if ((e = hipMemcpyAsync(ws, src, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
            return hip_fail(e, "copy to workspace");
        cur = ws;
    }
    for (int i = 0; i < nl; ++i) {
        void *out = ((nl - 1 - i) % 2 == 0) ? dst : ws;
        if (nck && launches[i].t0 % ck == 0) {
            const int s = launches[i].t0 / ck;
            if ((e = hipMemcpyAsync((char *)ckpt + s * bytes, cur, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
                return hip_fail(e, "copy checkpoint");
        }
        uint8_t *sel_t0 = sel ? sel + (size_t)launches[i].t0 * plane_set : nullptr;
        if ((e = enqueue_forward(plan, launches[i].k, cur, out, sel_t0, planes, H, W, r, dtype, stream,
                                 mode)) != hipSuccess)
            return hip_fail(e, "forward launch");
        cur = out;
    }
    return OSBF_SUCCESS;
}
}  // namespace

extern "C" {

osbf_status osbf_forward(const void *src, void *dst, int32_t planes, int32_t H, int32_t W,
                         osbf_dtype dtype, int32_t r, int32_t T, osbf_boundary boundary,
                         uint8_t *sel, void *ckpt, int32_t ck, void *ws, size_t ws_bytes,
                         void *stream) {
    return forward_impl(src, dst, planes, H, W, dtype, r, T, boundary, sel, ckpt, ck, ws, ws_bytes,
                        stream, 0);
}

}  // extern "C"

// Ping-pong iterate of osbf_forward_noalloc: one array per device, addressed
// through its device pointer (the name itself is a host-side stand-in).
static __device__ __align__(256) unsigned char scratch[OSBF_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64];  // per device, from hipGetSymbolAddress

// The current device's scratch address, looked up once per device.
osbf_status scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(OSBF_ERROR_UNSUPPORTED, "device %d: scratch kept for devices 0..63", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(OSBF_ERROR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return OSBF_SUCCESS;
}
}  // namespace

extern "C" {

osbf_status osbf_forward_noalloc(const void *src, void *dst, int32_t planes, int32_t H, int32_t W,
                                 osbf_dtype dtype, int32_t r, int32_t T, osbf_boundary boundary,
                                 void *stream) {
    g_last_error.clear();
    osbf_status st = check_sizes(planes, H, W, dtype, r, T);
    if (st != OSBF_SUCCESS) return st;
    const size_t bytes = (size_t)planes * H * W * elem_bytes(dtype);
    if (bytes > OSBF_NOALLOC_SCRATCH_BYTES)
        return fail(OSBF_ERROR_WORKSPACE,
                    "osbf_forward_noalloc: the image (%zu bytes) exceeds the %zu-byte scratch; "
                    "use osbf_forward with a workspace", bytes, (size_t)OSBF_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    if ((st = scratch_address(&ws)) != OSBF_SUCCESS) return st;
    return forward_impl(src, dst, planes, H, W, dtype, r, T, boundary, nullptr, nullptr, 0, ws,
                        OSBF_NOALLOC_SCRATCH_BYTES, stream, 0);
}

osbf_status osbf_forward_fast(const void *src, void *dst, int32_t planes, int32_t H, int32_t W,
                              osbf_dtype dtype, int32_t r, int32_t T, osbf_boundary boundary,
                              void *ws, size_t ws_bytes, void *stream) {
    return forward_impl(src, dst, planes, H, W, dtype, r, T, boundary, nullptr, nullptr, 0, ws,
                        ws_bytes, stream, 1);
}

osbf_status osbf_box_forward(const void *src, void *dst, int32_t planes, int32_t H, int32_t W,
                             osbf_dtype dtype, int32_t r, int32_t T, osbf_boundary boundary,
                             void *ws, size_t ws_bytes, void *stream_) {
    // the dedicated separable kernel for its radii; others (and planes too
    // wide for its 32-bit row offsets) take the box mode of the forward kernels
    if (!box_radius(r) || T == 0 || !stream_width_ok(W, (int)elem_bytes(dtype), r, stream_step(r)))
        return forward_impl(src, dst, planes, H, W, dtype, r, T, boundary, nullptr, nullptr, 0, ws,
                            ws_bytes, stream_, 2);
    g_last_error.clear();
    osbf_status st = check_sizes(planes, H, W, dtype, r, T);
    if (st != OSBF_SUCCESS) return st;
    if (boundary != OSBF_BOUNDARY_REPLICATE)
        return fail(OSBF_ERROR_INVALID_VALUE, "unknown boundary %d", (int)boundary);
    if (!src || !dst) return fail(OSBF_ERROR_INVALID_VALUE, "src and dst must be non-NULL");
    hipStream_t stream = (hipStream_t)stream_;
    const size_t bytes = (size_t)planes * H * W * elem_bytes(dtype);
    const bool need_ws = T >= 2 || src == dst;
    if (need_ws && (!ws || ws_bytes < bytes))
        return fail(OSBF_ERROR_WORKSPACE, "workspace of %zu bytes required, got %zu", bytes, ws ? ws_bytes : 0);
    hipError_t e;
    const void *cur = src;
    if (src == dst && (T % 2) == 1) {
        if ((e = hipMemcpyAsync(ws, src, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
            return hip_fail(e, "copy to workspace");
        cur = ws;
    }
    int tw = 0, step = 0;
    box_geometry(r, &tw, &step);
    const int tiles_x = (W + tw - 1) / tw;
    const int max_planes = std::max(1, (int)(((1LL << 31) - 1) / ((long long)tiles_x * H)));
    for (int t = 0; t < T; ++t) {
        void *out = ((T - 1 - t) % 2 == 0) ? dst : ws;
        for (int p0 = 0; p0 < planes; p0 += max_planes) {
            const size_t off = (size_t)p0 * H * W * elem_bytes(dtype);
            BoxLaunch a;
            a.src = (const char *)cur + off;
            a.dst = (char *)out + off;
            a.planes = std::min(max_planes, planes - p0);
            a.H = H; a.W = W; a.r = r;
            a.tw = tw; a.th = 0; a.tiles_x = tiles_x; a.tiles_y = 0;
            if ((e = launch_box((int)dtype, a, stream)) != hipSuccess) return hip_fail(e, "box filter launch");
        }
        cur = out;
    }
    return OSBF_SUCCESS;
}

size_t osbf_backward_workspace_size(int32_t planes, int32_t H, int32_t W, int32_t r, int32_t T,
                                    int32_t ck) {
    if (check_sizes(planes, H, W, OSBF_F32, r, T) != OSBF_SUCCESS || ck < 0) return (size_t)-1;
    if (T == 0 || r == 0) return 0;
    const size_t P = (size_t)planes * H * W;
    size_t n = P * sizeof(float);                        // gradient ping-pong
    if (ck > 0) n += 2 * P * sizeof(float) + (size_t)std::min(ck, T) * P;  // recompute buffers, maps
    if (r > kAdjointLdsMaxR)  // the two-pass adjoint's planes, after the rest (256-byte aligned)
        n = (n + 255) / 256 * 256 + adjoint_global_ws_bytes(planes, H, W, r);
    return n;
}

osbf_status osbf_backward(const float *grad_out, float *grad_in, int32_t planes, int32_t H,
                          int32_t W, int32_t r, int32_t T, osbf_boundary boundary,
                          const uint8_t *sel, const float *ckpt, int32_t ck, void *ws,
                          size_t ws_bytes, void *stream_) {
    g_last_error.clear();
    osbf_status st = check_sizes(planes, H, W, OSBF_F32, r, T);
    if (st != OSBF_SUCCESS) return st;
    if (boundary != OSBF_BOUNDARY_REPLICATE)
        return fail(OSBF_ERROR_INVALID_VALUE, "unknown boundary %d", (int)boundary);
    if (!grad_out || !grad_in) return fail(OSBF_ERROR_INVALID_VALUE, "gradients must be non-NULL");
    hipStream_t stream = (hipStream_t)stream_;
    const size_t P = (size_t)planes * H * W;
    const size_t gbytes = P * sizeof(float);
    hipError_t e;
    if (T == 0 || r == 0) {  // identity map
        if (grad_in != grad_out &&
            (e = hipMemcpyAsync(grad_in, grad_out, gbytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
            return hip_fail(e, "copy");
        return OSBF_SUCCESS;
    }
    if ((sel == nullptr) == (ckpt == nullptr))
        return fail(OSBF_ERROR_INVALID_VALUE, "pass exactly one of sel (all maps) or ckpt (checkpoints)");
    if (ckpt && ck < 1) return fail(OSBF_ERROR_INVALID_VALUE, "checkpoint interval %d < 1", ck);
    const size_t need = osbf_backward_workspace_size(planes, H, W, r, T, ckpt ? ck : 0);
    if (!ws || ws_bytes < need)
        return fail(OSBF_ERROR_WORKSPACE, "workspace of %zu bytes required, got %zu", need, ws ? ws_bytes : 0);

    BwdLaunch b{};
    const bool global_pass = r > kAdjointLdsMaxR;  // beyond the LDS-resident kernels
    float *wglob = nullptr;
    if (global_pass) {
        const size_t base = osbf_backward_workspace_size(planes, H, W, r, T, ckpt ? ck : 0) -
                            adjoint_global_ws_bytes(planes, H, W, r);
        wglob = (float *)((char *)ws + base);
        b.tw = W; b.th = H;
    } else if (!adjoint_tile(r, W, &b)) {
        return fail(OSBF_ERROR_UNSUPPORTED, "radius %d does not fit the device's LDS", r);
    }
    b.H = H; b.W = W; b.r = r;
    b.tiles_x = (W + b.tw - 1) / b.tw;
    b.tiles_y = (H + b.th - 1) / b.th;
    const int max_planes = global_pass ? 65535
                                       : std::max(1, (int)(((1LL << 31) - 1) / ((long long)b.tiles_x * b.tiles_y)));

    float *wsg = (float *)ws;
    float *f1 = nullptr, *f2 = nullptr;
    uint8_t *wsel = nullptr;
    if (ckpt) {
        f1 = wsg + P;
        f2 = f1 + P;
        wsel = (uint8_t *)(f2 + P);
    }
    // sweep t = T-1 .. 0; the last one (t = 0) writes grad_in
    const float *gin = grad_out;
    if (grad_out == grad_in && (T % 2) == 1) {
        if ((e = hipMemcpyAsync(wsg, grad_out, gbytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
            return hip_fail(e, "copy to workspace");
        gin = wsg;
    }
    auto adjoint = [&](int t, const uint8_t *sel_t) -> hipError_t {
        float *gout = (t % 2 == 0) ? grad_in : wsg;
        for (int p0 = 0; p0 < planes; p0 += max_planes) {
            const size_t off = (size_t)p0 * H * W;
            b.planes = std::min(max_planes, planes - p0);
            b.gnext = gin + off;
            b.sel = sel_t + off;
            b.g = gout + off;
            hipError_t err = global_pass ? launch_adjoint_global(b, wglob, stream) : launch_adjoint(b, stream);
            if (err != hipSuccess) return err;
        }
        gin = gout;
        return hipSuccess;
    };

    if (sel) {
        for (int t = T - 1; t >= 0; --t)
            if ((e = adjoint(t, sel + (size_t)t * P)) != hipSuccess) return hip_fail(e, "adjoint launch");
        return OSBF_SUCCESS;
    }
    // Checkpoint mode: recompute each segment's maps with the forward's own
    // launches (bit-identical maps), then run that segment's adjoints.
    const Plan plan = choose_plan(planes, H, W, r, T, OSBF_F32);
    if (!plan.tw) return fail(OSBF_ERROR_UNSUPPORTED, "radius %d does not fit the device's LDS", r);
    const std::vector<Launch> launches = make_launches(T, ck, plan.k);
    const int nseg = (T + ck - 1) / ck;
    for (int sidx = nseg - 1; sidx >= 0; --sidx) {
        const int s0 = sidx * ck, s1 = std::min(T, s0 + ck);
        const void *cur = ckpt + (size_t)sidx * P;
        bool use_f1 = true;
        for (const Launch &L : launches) {
            if (L.t0 < s0 || L.t0 >= s1) continue;
            float *out = use_f1 ? f1 : f2;
            use_f1 = !use_f1;
            if ((e = enqueue_forward(plan, L.k, cur, out, wsel + (size_t)(L.t0 - s0) * P, planes, H, W,
                                     r, OSBF_F32, stream)) != hipSuccess)
                return hip_fail(e, "forward recompute");
            cur = out;
        }
        for (int t = s1 - 1; t >= s0; --t)
            if ((e = adjoint(t, wsel + (size_t)(t - s0) * P)) != hipSuccess) return hip_fail(e, "adjoint launch");
    }
    return OSBF_SUCCESS;
}

osbf_status osbf_forward_plan(int32_t planes, int32_t H, int32_t W, osbf_dtype dtype,
                              int32_t r, int32_t T, int32_t ck, int32_t *tile_w,
                              int32_t *tile_h, int32_t *fused, int32_t *launches) {
    g_last_error.clear();
    osbf_status st = check_sizes(planes, H, W, dtype, r, T);
    if (st != OSBF_SUCCESS) return st;
    if (!tile_w || !tile_h || !fused || !launches)
        return fail(OSBF_ERROR_INVALID_VALUE, "output pointers must be non-NULL");
    if (T == 0 || r == 0) {
        *tile_w = *tile_h = *fused = *launches = 0;
        return OSBF_SUCCESS;
    }
    const Plan plan = choose_plan(planes, H, W, r, T, (int)dtype);
    if (!plan.tw)
        return fail(OSBF_ERROR_UNSUPPORTED, "radius %d does not fit the device's LDS", r);
    *tile_w = plan.tw;
    *tile_h = plan_rows(plan, r);
    *fused = plan.k;
    *launches = (int32_t)make_launches(T, ck > 0 ? ck : 0, plan.k).size();
    return OSBF_SUCCESS;
}

}  // extern "C"

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct BatchImagePlan {
    int rounds = 0;
    int tw = 0, th = 0;  // strip width, rows per work item
    size_t side_ws = 0;  // radius without a batched kernel: osbf_forward's workspace
};

// Per-image plans of a batch (row-streaming work items, one sweep per round)
// and the table sizes.
struct BatchLayout {
    std::vector<BatchImagePlan> img;
    int rounds = 0, maxr = 0;
    int64_t max_items = 0, total_items = 0;
    size_t descs_off = 0, items_off = 0, counts_off = 0, bufs_off = 0, total = 0;
    std::vector<size_t> buf_off;
    int identity = 0;
    int side = 0;  // images of a radius without a batched kernel (osbf_forward's launches)
};

// Rows per work item: long enough that the r halo rows a chunk recomputes
// stay small, short enough that a round has many items to balance (the
// 256-image mixed batch: 32 rows 324 K, 64 rows 340 K, 128 rows 330 K
// MPix*it/s).
constexpr int kBatchRows = 64;

// Per round, two kernel classes (radius above kBatchLeanMaxR, and up to it),
// each with the offsets of its 8 XCD bins in the round's item list plus the
// end.
constexpr int kBinTable = 2 * 9;

// Relative cost of one lane-row of a work item by radius (time per sweep of
// the 128-lane streaming kernel on 3x2048^2 times its strip width, MI355X;
// the radii in between take the next larger entry).
double item_row_cost(int r) {
    return r <= 1 ? 2.72 : r <= 2 ? 2.89 : r <= 5 ? 2.90 : r <= 8 ? 3.16 : r <= 10 ? 3.2 : 4.3;
}

// Static LPT partition of one kernel class's items of a round over the 8 XCD
// bins.  Consecutive items of an image (neighbouring strips, then chunks)
// form groups of bounded cost so that halo rows and columns meet in one L2;
// groups go, largest first, to the bin with the least load; each bin lists
// its groups by decreasing per-item cost for the workgroups' round-robin.
struct BinGroup { double cost; int img, w0, w1; double item_cost; };

void lpt_bins(std::vector<BinGroup> &groups, std::vector<uint2> &out, int *offs) {
    std::stable_sort(groups.begin(), groups.end(),
                     [](const BinGroup &a, const BinGroup &b) { return a.cost > b.cost; });
    std::vector<std::vector<const BinGroup *>> bins(8);
    double load[8] = {0};
    for (const BinGroup &g : groups) {
        int best = 0;
        for (int b = 1; b < 8; ++b)
            if (load[b] < load[best]) best = b;
        load[best] += g.cost;
        bins[best].push_back(&g);
    }
    for (int b = 0; b < 8; ++b) {
        std::stable_sort(bins[b].begin(), bins[b].end(),
                         [](const BinGroup *x, const BinGroup *y) { return x->item_cost > y->item_cost; });
        offs[b] = (int)out.size();
        for (const BinGroup *g : bins[b])
            for (int w = g->w0; w < g->w1; ++w) out.push_back(make_uint2((unsigned)g->img, (unsigned)w));
    }
    offs[8] = (int)out.size();
}

// Rows per batched work item for radius r: an override (tuning), else the
// autotuned value for this device model, else kBatchRows.
int batch_rows(int r, int dtype, const int *rows_override) {
    if (rows_override && rows_override[r] > 0) return rows_override[r];
    const std::string model = current_model();
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_file_read_locked();
    auto it = g_tune_batch.find(std::make_tuple(model, dtype, r));
    return it != g_tune_batch.end() ? it->second : kBatchRows;
}

osbf_status batch_layout(const osbf_image *imgs, int n, osbf_dtype dtype, BatchLayout *L,
                         const int *rows_override = nullptr) {
    if (n < 0 || (n > 0 && !imgs)) return fail(OSBF_ERROR_INVALID_VALUE, "bad image list");
    if (!valid_dtype(dtype)) return fail(OSBF_ERROR_INVALID_VALUE, "unknown dtype %d", (int)dtype);
    L->img.resize(n);
    L->buf_off.resize(n);
    std::vector<int64_t> per_round;
    for (int j = 0; j < n; ++j) {
        const osbf_image &m = imgs[j];
        osbf_status st = check_sizes(m.planes, m.height, m.width, dtype, m.radius, m.iterations);
        if (st != OSBF_SUCCESS) return fail(st, "image %d: %s", j, g_last_error.c_str());
        if (!m.src || !m.dst) return fail(OSBF_ERROR_INVALID_VALUE, "image %d: NULL pointer", j);
        if (m.src == m.dst) return fail(OSBF_ERROR_INVALID_VALUE, "image %d: src and dst must differ", j);
        for (int side = 0; side < 2; ++side) {
            const int64_t ld = side ? m.dst_row_stride : m.src_row_stride;
            const int64_t ps = side ? m.dst_plane_stride : m.src_plane_stride;
            const int64_t rows = ld ? ld : m.width;
            if (ld < 0 || (ld && ld < m.width) || ld > INT32_MAX)
                return fail(OSBF_ERROR_INVALID_VALUE, "image %d: %s row stride %lld (width %d)", j,
                            side ? "dst" : "src", (long long)ld, m.width);
            if (ps < 0 || (ps && m.planes > 1 && ps < (int64_t)m.height * rows))
                return fail(OSBF_ERROR_INVALID_VALUE, "image %d: %s plane stride %lld < height x row stride", j,
                            side ? "dst" : "src", (long long)ps);
        }
        BatchImagePlan &b = L->img[j];
        if (m.radius == 0 || m.iterations == 0) {
            L->identity++;
            continue;
        }
        if (!fixed_radius(m.radius)) {
            // no batched kernel for this radius: osbf_batched runs the image
            // through osbf_forward's own launches, on contiguous planes only
            auto dense = [&](int64_t ld, int64_t ps) {
                const int64_t l = ld ? ld : m.width;
                return (l == m.width || m.height == 1) &&
                       (m.planes == 1 || !ps || ps == (int64_t)m.height * m.width);
            };
            if (!dense(m.src_row_stride, m.src_plane_stride) || !dense(m.dst_row_stride, m.dst_plane_stride))
                return fail(OSBF_ERROR_UNSUPPORTED,
                            "image %d: radius %d has no batched kernel; its single-image path needs contiguous "
                            "planes", j, m.radius);
            b.side_ws = osbf_forward_workspace_size(m.planes, m.height, m.width, dtype, m.radius, m.iterations);
            if (b.side_ws == (size_t)-1) return fail(OSBF_ERROR_INVALID_VALUE, "image %d: bad size", j);
            L->side++;
            continue;
        }
        const int r = m.radius, step = stream_step(r);
        b.tw = ((batched_lanes() - 2 * r) / r) * r;
        b.th = (std::min(m.height, batch_rows(r, (int)dtype, rows_override)) + step - 1) / step * step;
        const int64_t ld_max = std::max<int64_t>(m.width, std::max(m.src_row_stride, m.dst_row_stride));
        if (!stream_width_ok((int)ld_max, (int)elem_bytes(dtype), r, b.th))
            return fail(OSBF_ERROR_UNSUPPORTED, "image %d: row of %lld elements too long for the batched kernel", j,
                        (long long)ld_max);
        b.rounds = m.iterations;
        L->maxr = std::max(L->maxr, r);
        const int64_t tiles = (int64_t)((m.width + b.tw - 1) / b.tw) * ((m.height + b.th - 1) / b.th);
        const int64_t items = tiles * m.planes;
        if ((int)per_round.size() < b.rounds) per_round.resize(b.rounds, 0);
        for (int r = 0; r < b.rounds; ++r) per_round[r] += items;
        L->total_items += items * b.rounds;
        L->rounds = std::max(L->rounds, b.rounds);
    }
    for (int64_t c : per_round) L->max_items = std::max(L->max_items, c);
    if (L->max_items > (int64_t)INT32_MAX) return fail(OSBF_ERROR_UNSUPPORTED, "batch too large");
    size_t off = 0;
    L->descs_off = off;
    off = align256(off + (size_t)L->rounds * n * sizeof(FwdLaunch));
    L->items_off = off;
    off = align256(off + (size_t)L->rounds * L->max_items * sizeof(uint2));
    L->counts_off = off;  // per round and kernel class: 9 bin offsets (one bin per XCD)
    off = align256(off + (size_t)kBinTable * std::max(L->rounds, 1) * sizeof(int));
    L->bufs_off = off;
    for (int j = 0; j < n; ++j) {
        L->buf_off[j] = off;
        if (L->img[j].rounds >= 2)
            off = align256(off + (size_t)imgs[j].planes * imgs[j].height * imgs[j].width * elem_bytes(dtype));
        else if (L->img[j].side_ws)
            off = align256(off + L->img[j].side_ws);
    }
    L->total = off;
    return OSBF_SUCCESS;
}


}  // namespace

extern "C" {

size_t osbf_batched_workspace_size(const osbf_image *imgs, int32_t n, osbf_dtype dtype) {
    BatchLayout L;
    if (batch_layout(imgs, n, dtype, &L) != OSBF_SUCCESS) return (size_t)-1;
    return L.total;
}

static osbf_status batched_prepare_impl(const osbf_image *imgs, int32_t n, osbf_dtype dtype,
                                       osbf_boundary boundary, void *ws, size_t ws_bytes,
                                       osbf_batch *batch, void *stream_, const int *rows_override) {
    g_last_error.clear();
    if (!batch) return fail(OSBF_ERROR_INVALID_VALUE, "batch must be non-NULL");
    if (boundary != OSBF_BOUNDARY_REPLICATE)
        return fail(OSBF_ERROR_INVALID_VALUE, "unknown boundary %d", (int)boundary);
    BatchLayout L;
    osbf_status st = batch_layout(imgs, n, dtype, &L, rows_override);
    if (st != OSBF_SUCCESS) return st;
    if (L.total && (!ws || ws_bytes < L.total))
        return fail(OSBF_ERROR_WORKSPACE, "workspace of %zu bytes required, got %zu", L.total, ws ? ws_bytes : 0);
    hipStream_t stream = (hipStream_t)stream_;
    // host tables
    std::vector<FwdLaunch> descs((size_t)L.rounds * n);
    std::vector<uint2> items((size_t)L.rounds * L.max_items);
    // images in decreasing cost order (radius) for the work lists
    std::vector<int> order;
    for (int j = 0; j < n; ++j)
        if (L.img[j].rounds) order.push_back(j);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return imgs[a].radius > imgs[b].radius; });
    for (int j = 0; j < n; ++j) {
        const BatchImagePlan &b = L.img[j];
        const osbf_image &m = imgs[j];
        void *buf = (char *)ws + L.buf_off[j];
        const void *cur = m.src;
        int cur_ld = (int)m.src_row_stride;   // the workspace iterate is contiguous (0)
        long long cur_ps = m.src_plane_stride;
        for (int r = 0; r < b.rounds; ++r) {
            const bool to_dst = (b.rounds - 1 - r) % 2 == 0;
            void *out = to_dst ? m.dst : buf;
            FwdLaunch &a = descs[(size_t)r * n + j];
            a.src = cur;
            a.dst = out;
            a.src_ld = cur_ld;
            a.src_ps = cur_ps;
            a.dst_ld = to_dst ? (int)m.dst_row_stride : 0;
            a.dst_ps = to_dst ? m.dst_plane_stride : 0;
            cur_ld = a.dst_ld;
            cur_ps = a.dst_ps;
            a.sel = nullptr;
            a.sel_stride = 0;
            a.planes = m.planes;
            a.H = m.height; a.W = m.width; a.r = m.radius;
            a.k = 1;
            a.tw = b.tw; a.th = b.th;
            a.tiles_x = (m.width + b.tw - 1) / b.tw;
            a.tiles_y = (m.height + b.th - 1) / b.th;
            a.pitch = a.arr = 0;
            a.geom = GEOM_S128;
            cur = out;
        }
    }
    // a round's items per kernel class (radius above kBatchLeanMaxR, and up
    // to it), each split over the 8 XCD bins by cost
    bool any_big = false, any_small = false;
    int lean_maxr = 0;
    for (int j : order) {
        (imgs[j].radius > kBatchLeanMaxR ? any_big : any_small) = true;
        if (imgs[j].radius <= kBatchLeanMaxR) lean_maxr = std::max(lean_maxr, (int)imgs[j].radius);
    }
    std::vector<int> counts((size_t)kBinTable * std::max(L.rounds, 1), 0);
    for (int r = 0; r < L.rounds; ++r) {
        std::vector<uint2> list;
        list.reserve((size_t)L.max_items);
        for (int cls = 0; cls < 2; ++cls) {
            double total = 0;
            for (int j : order) {
                if (r >= L.img[j].rounds || (imgs[j].radius > kBatchLeanMaxR) != (cls == 0)) continue;
                const FwdLaunch &a = descs[(size_t)r * n + j];
                total += (double)a.tiles_x * a.tiles_y * a.planes * (a.th + a.r) * item_row_cost(a.r);
            }
            const double cap = std::max(total / (8.0 * 32.0), 1e-9);  // at least ~32 groups per bin
            std::vector<BinGroup> groups;
            for (int j : order) {
                if (r >= L.img[j].rounds || (imgs[j].radius > kBatchLeanMaxR) != (cls == 0)) continue;
                const FwdLaunch &a = descs[(size_t)r * n + j];
                const int cnt = a.tiles_x * a.tiles_y * a.planes;
                const double ic = (a.th + a.r) * item_row_cost(a.r);
                const int per = std::max(1, (int)(cap / ic));
                for (int w = 0; w < cnt; w += per) {
                    const int w1 = std::min(cnt, w + per);
                    groups.push_back(BinGroup{ic * (w1 - w), j, w, w1, ic});
                }
            }
            int *offs = counts.data() + (size_t)kBinTable * r + 9 * cls;
            lpt_bins(groups, list, offs);
        }
        std::copy(list.begin(), list.end(), items.begin() + (size_t)r * L.max_items);
    }
    hipError_t e;
    if (L.rounds) {
        if ((e = hipMemcpyAsync((char *)ws + L.descs_off, descs.data(), descs.size() * sizeof(FwdLaunch),
                                hipMemcpyHostToDevice, stream)) != hipSuccess ||
            (e = hipMemcpyAsync((char *)ws + L.items_off, items.data(), items.size() * sizeof(uint2),
                                hipMemcpyHostToDevice, stream)) != hipSuccess ||
            (e = hipMemcpyAsync((char *)ws + L.counts_off, counts.data(), (size_t)kBinTable * L.rounds * sizeof(int),
                                hipMemcpyHostToDevice, stream)) != hipSuccess)
            return hip_fail(e, "upload batch tables");
        // the host vectors go out of scope: wait for the copies
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, "synchronize");
    }
    int slots = 0, slots_small = 0;
    if (L.rounds && any_big && (e = batched_slots((int)dtype, L.maxr, &slots)) != hipSuccess)
        return hip_fail(e, "occupancy");
    if (L.rounds && any_small && (e = batched_slots((int)dtype, lean_maxr, &slots_small)) != hipSuccess)
        return hip_fail(e, "occupancy");
    const int64_t g = std::min<int64_t>(L.max_items, std::max(slots, 1));
    const int64_t gs = std::min<int64_t>(L.max_items, std::max(slots_small, 1));
    memset(batch, 0, sizeof *batch);
    batch->n = n;
    batch->dtype = dtype;
    batch->rounds = L.rounds;
    batch->grid = (int)std::max<int64_t>(8, (g + 7) / 8 * 8);
    batch->max_items = L.max_items;
    batch->total_items = L.total_items;
    batch->ws = ws;
    batch->descs_off = L.descs_off;
    batch->items_off = L.items_off;
    batch->counts_off = L.counts_off;
    batch->identity = L.identity;
    batch->reserved[2] = L.side;                // images left to osbf_forward's launches (osbf_batched)
    batch->reserved[0] = any_big ? L.maxr : 0;  // class of the launches above the lean radii (0: none)
    batch->reserved[1] = any_small ? (int)std::max<int64_t>(8, (gs + 7) / 8 * 8) : 0;  // grid of the lean launches
    batch->reserved[3] = any_small ? lean_maxr : 0;  // class of the lean launches
    // identity images are copied at launch: remember them in the tables is
    // not needed; the launch re-reads the host list through the caller.
    return OSBF_SUCCESS;
}

osbf_status osbf_batched_prepare(const osbf_image *imgs, int32_t n, osbf_dtype dtype,
                                 osbf_boundary boundary, void *ws, size_t ws_bytes,
                                 osbf_batch *batch, void *stream_) {
    return batched_prepare_impl(imgs, n, dtype, boundary, ws, ws_bytes, batch, stream_, nullptr);
}

osbf_status osbf_batched_launch(const osbf_batch *batch, void *stream_) {
    g_last_error.clear();
    if (!batch) return fail(OSBF_ERROR_INVALID_VALUE, "batch must be non-NULL");
    if (batch->identity)
        return fail(OSBF_ERROR_UNSUPPORTED, "batch has identity images (r = 0 or T = 0): use osbf_batched");
    if (batch->reserved[2])
        return fail(OSBF_ERROR_UNSUPPORTED, "batch has images of a radius without a batched kernel: use osbf_batched");
    hipStream_t stream = (hipStream_t)stream_;
    const FwdLaunch *descs = (const FwdLaunch *)((const char *)batch->ws + batch->descs_off);
    const uint2 *items = (const uint2 *)((const char *)batch->ws + batch->items_off);
    const int *counts = (const int *)((const char *)batch->ws + batch->counts_off);
    for (int r = 0; r < batch->rounds; ++r) {
        const FwdLaunch *d = descs + (size_t)r * batch->n;
        const uint2 *it = items + (size_t)r * batch->max_items;
        hipError_t e = hipSuccess;
        const int *offs = counts + (size_t)kBinTable * r;
        if (batch->reserved[0])  // radius above kBatchLeanMaxR
            e = launch_batched_round(batch->dtype, batch->reserved[0], d, it, offs, batch->grid, stream);
        if (e == hipSuccess && batch->reserved[1])  // the lean radii, after the others in the list
            e = launch_batched_round(batch->dtype, batch->reserved[3], d, it, offs + 9, batch->reserved[1], stream);
        if (e != hipSuccess) return hip_fail(e, "batched launch");
    }
    return OSBF_SUCCESS;
}

osbf_status osbf_batched(const osbf_image *imgs, int32_t n, osbf_dtype dtype, osbf_boundary boundary,
                         void *ws, size_t ws_bytes, void *stream_) {
    osbf_batch b;
    osbf_status st = osbf_batched_prepare(imgs, n, dtype, boundary, ws, ws_bytes, &b, stream_);
    if (st != OSBF_SUCCESS) return st;
    hipStream_t stream = (hipStream_t)stream_;
    BatchLayout L;  // the workspace slices of the images left to osbf_forward
    if (b.reserved[2] && (st = batch_layout(imgs, n, dtype, &L)) != OSBF_SUCCESS) return st;
    for (int j = 0; j < n; ++j) {
        const osbf_image &m = imgs[j];
        if (m.radius > 0 && m.iterations > 0 && !fixed_radius(m.radius)) {
            const size_t bytes = L.img[j].side_ws;
            st = osbf_forward(m.src, m.dst, m.planes, m.height, m.width, dtype, m.radius, m.iterations, boundary,
                              nullptr, nullptr, 0, bytes ? (char *)ws + L.buf_off[j] : nullptr, bytes, stream_);
            if (st != OSBF_SUCCESS) return st;
            continue;
        }
        if (m.radius == 0 || m.iterations == 0) {
            const size_t es = elem_bytes(dtype), row = (size_t)m.width * es;
            const size_t sld = m.src_row_stride ? (size_t)m.src_row_stride * es : row;
            const size_t dld = m.dst_row_stride ? (size_t)m.dst_row_stride * es : row;
            const size_t sps = m.src_plane_stride ? (size_t)m.src_plane_stride * es : sld * m.height;
            const size_t dps = m.dst_plane_stride ? (size_t)m.dst_plane_stride * es : dld * m.height;
            hipError_t e = hipSuccess;
            if (sld == row && dld == row && sps == row * m.height && dps == row * m.height) {
                e = hipMemcpyAsync(m.dst, m.src, row * m.height * m.planes, hipMemcpyDeviceToDevice, stream);
            } else {
                for (int p = 0; p < m.planes && e == hipSuccess; ++p)
                    e = hipMemcpy2DAsync((char *)m.dst + p * dps, dld, (const char *)m.src + p * sps, sld, row,
                                         m.height, hipMemcpyDeviceToDevice, stream);
            }
            if (e != hipSuccess) return hip_fail(e, "copy");
        }
    }
    b.identity = 0;
    b.reserved[2] = 0;
    return osbf_batched_launch(&b, stream_);
}


// Candidate rows per batched work item (the 256-image workload measured 32 /
// 64 / 128 rows within 5% of each other with one item shape for all radii).
static const int kBatchRowCands[] = {32, 64, 128};

size_t osbf_batched_autotune_workspace_size(const osbf_image *imgs, int32_t n, osbf_dtype dtype) {
    // the shortest candidate items give the longest item tables
    int rows[OSBF_MAX_RADIUS + 1];
    for (int &v : rows) v = kBatchRowCands[0];
    BatchLayout L;
    if (batch_layout(imgs, n, dtype, &L, rows) != OSBF_SUCCESS) return (size_t)-1;
    BatchLayout D;
    if (batch_layout(imgs, n, dtype, &D) != OSBF_SUCCESS) return (size_t)-1;
    return std::max(L.total, D.total);
}

osbf_status osbf_batched_autotune(const osbf_image *imgs, int32_t n, osbf_dtype dtype, void *ws,
                                  size_t ws_bytes, void *stream_, int32_t *rows_out) {
    g_last_error.clear();
    const size_t need = osbf_batched_autotune_workspace_size(imgs, n, dtype);
    if (need == (size_t)-1) {
        BatchLayout L;
        return batch_layout(imgs, n, dtype, &L);  // reports the error
    }
    if (need && (!ws || ws_bytes < need))
        return fail(OSBF_ERROR_WORKSPACE, "workspace of %zu bytes required, got %zu", need, ws ? ws_bytes : 0);
    hipStream_t stream = (hipStream_t)stream_;
    int cur[OSBF_MAX_RADIUS + 1] = {0};
    bool present[OSBF_MAX_RADIUS + 1] = {false};
    for (int j = 0; j < n; ++j)
        if (imgs[j].radius > 0 && imgs[j].iterations > 0) present[imgs[j].radius] = true;
    for (int r = 1; r <= OSBF_MAX_RADIUS; ++r)
        if (present[r]) cur[r] = batch_rows(r, (int)dtype, nullptr);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // best of three timed replays of the whole batch under a candidate
    auto measure = [&](const int *rows, double *ms_out) -> osbf_status {
        osbf_batch b;
        osbf_status st = batched_prepare_impl(imgs, n, dtype, OSBF_BOUNDARY_REPLICATE, ws, ws_bytes, &b, stream_,
                                              rows);
        if (st != OSBF_SUCCESS) return st;
        b.identity = 0;     // identity images take no kernel time
        b.reserved[2] = 0;  // nor do they count here the images left to osbf_forward
        double best = 1e300;
        for (int rep = 0; rep < 4; ++rep) {
            if ((e = hipEventRecord(e0, stream)) != hipSuccess) return hip_fail(e, "event");
            if ((st = osbf_batched_launch(&b, stream_)) != OSBF_SUCCESS) return st;
            if ((e = hipEventRecord(e1, stream)) != hipSuccess) return hip_fail(e, "event");
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "synchronize");
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return hip_fail(e, "event");
            if (rep > 0) best = std::min(best, (double)ms);  // the first replay warms up
        }
        *ms_out = best;
        return OSBF_SUCCESS;
    };
    osbf_status st = e == hipSuccess ? OSBF_SUCCESS : hip_fail(e, "event");
    double best_ms = 0;
    if (st == OSBF_SUCCESS) st = measure(cur, &best_ms);
    // one radius at a time, the others at their current choice; a candidate
    // must beat the incumbent by 3% (replays vary by a few percent)
    for (int r = 1; r <= OSBF_MAX_RADIUS && st == OSBF_SUCCESS; ++r) {
        if (!present[r]) continue;
        for (int rows : kBatchRowCands) {
            if (rows == cur[r] || st != OSBF_SUCCESS) continue;
            int cand[OSBF_MAX_RADIUS + 1];
            std::copy(cur, cur + OSBF_MAX_RADIUS + 1, cand);
            cand[r] = rows;
            double ms = 0;
            st = measure(cand, &ms);
            if (st == OSBF_SUCCESS && ms < 0.97 * best_ms) {
                best_ms = ms;
                cur[r] = rows;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != OSBF_SUCCESS) return st;
    const std::string model = current_model();
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        tune_file_read_locked();
        for (int r = 1; r <= OSBF_MAX_RADIUS; ++r)
            if (present[r]) g_tune_batch[std::make_tuple(model, (int)dtype, r)] = cur[r];
        tune_file_write_locked();
    }
    if (rows_out)
        for (int r = 0; r <= OSBF_MAX_RADIUS; ++r) rows_out[r] = present[r] ? cur[r] : 0;
    return OSBF_SUCCESS;
}

size_t osbf3d_forward_workspace_size(int32_t vols, int32_t D, int32_t H, int32_t W, int32_t r,
                                     int32_t T) {
    if (vols < 1 || D < 1 || H < 1 || W < 1 || r < 0 || r > OSBF3D_MAX_RADIUS || T < 0) return (size_t)-1;
    if (T == 0 || r == 0) return 0;
    return (size_t)vols * D * H * W * sizeof(float);
}

osbf_status osbf3d_forward(const float *src, float *dst, int32_t vols, int32_t D, int32_t H,
                           int32_t W, int32_t r, int32_t T, uint8_t *sel, void *ws,
                           size_t ws_bytes, void *stream_) {
    g_last_error.clear();
    if (vols < 1 || D < 1 || H < 1 || W < 1)
        return fail(OSBF_ERROR_INVALID_VALUE, "volumes, depth, height and width must be >= 1 (got %d, %d, %d, %d)",
                    vols, D, H, W);
    if ((long long)D * H * W > (1LL << 40)) return fail(OSBF_ERROR_INVALID_VALUE, "volume too large");
    if (r < 0) return fail(OSBF_ERROR_INVALID_VALUE, "radius %d < 0", r);
    if (r > OSBF3D_MAX_RADIUS)
        return fail(OSBF_ERROR_UNSUPPORTED, "volume radius %d above %d", r, OSBF3D_MAX_RADIUS);
    if (T < 0) return fail(OSBF_ERROR_INVALID_VALUE, "iterations %d < 0", T);
    if (!src || !dst) return fail(OSBF_ERROR_INVALID_VALUE, "src and dst must be non-NULL");
    hipStream_t stream = (hipStream_t)stream_;
    const size_t nvox = (size_t)vols * D * H * W;
    const size_t bytes = nvox * sizeof(float);
    hipError_t e;
    if (T == 0 || r == 0) {
        if (src != dst && (e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
            return hip_fail(e, "copy");
        if (sel && T > 0 && (e = hipMemsetAsync(sel, 0, (size_t)T * nvox, stream)) != hipSuccess)
            return hip_fail(e, "memset sel");
        return OSBF_SUCCESS;
    }
    if ((T >= 2 || src == dst) && (!ws || ws_bytes < bytes))
        return fail(OSBF_ERROR_WORKSPACE, "workspace of %zu bytes required, got %zu", bytes, ws ? ws_bytes : 0);

    Fwd3dLaunch a;
    int th;
    a.threads = fwd3d_threads(r);
    fwd3d_geometry(r, a.threads, &a.tw, &th);
    a.vols = vols; a.D = D; a.H = H; a.W = W; a.r = r;
    a.tiles_x = (W + a.tw - 1) / a.tw;
    a.tiles_y = (H + th - 1) / th;
    const long long layer = (long long)a.tiles_x * a.tiles_y * vols;
    // slice chunks: a radius-dependent number of slices each (a chunk pays
    // 2r warm-up slices, so longer chunks at larger r; measured on 256^3:
    // r=1 16, r=2 32, r=3 and 4 48 slices, r=4 114 K MVox*it/s against 98 K
    // at 32), more chunks only to fill the device (OSBF_3D_SLICES=n forces n
    // slices per chunk: tests, sweeps)
    const int zt = r == 1 ? 16 : r == 2 ? 32 : 48;
    long long chunks = std::max(1LL, std::min((long long)(D + zt - 1) / zt, (2048 + layer - 1) / layer));
    if (const char *env = getenv("OSBF_3D_SLICES")) {
        const int zs = atoi(env);
        if (zs > 0) chunks = (D + zs - 1) / zs;
    }
    a.zc = (int)((D + chunks - 1) / chunks);
    a.chunks = (D + a.zc - 1) / a.zc;
    if (layer * a.chunks >= (1LL << 31)) return fail(OSBF_ERROR_INVALID_VALUE, "too many tiles");

    const float *cur = src;
    if (src == dst && (T % 2) == 1) {
        if ((e = hipMemcpyAsync(ws, src, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
            return hip_fail(e, "copy to workspace");
        cur = (const float *)ws;
    }
    for (int t = 0; t < T; ++t) {
        float *out = ((T - 1 - t) % 2 == 0) ? dst : (float *)ws;
        a.src = cur;
        a.dst = out;
        a.sel = sel ? sel + (size_t)t * nvox : nullptr;
        if ((e = launch_forward3d(a, stream)) != hipSuccess) return hip_fail(e, "volume launch");
        cur = out;
    }
    return OSBF_SUCCESS;
}


size_t osbf_gaussian_workspace_size(int32_t planes, int32_t H, int32_t W, int32_t r, int32_t T) {
    if (planes < 1 || H < 1 || W < 1 || r < 0 || r > OSBF_GAUSS_MAX_RADIUS || T < 0) return (size_t)-1;
    if (T == 0 || r == 0) return 0;
    return (size_t)planes * H * W * sizeof(float);
}

osbf_status osbf_gaussian_forward(const float *src, float *dst, int32_t planes, int32_t H, int32_t W,
                                  int32_t r, float sigma, int32_t T, uint8_t *sel, void *ws,
                                  size_t ws_bytes, void *stream_) {
    g_last_error.clear();
    osbf_status st = check_sizes(planes, H, W, OSBF_F32, std::min(r, (int32_t)OSBF_MAX_RADIUS), T);
    if (st != OSBF_SUCCESS) return st;
    if (r > OSBF_GAUSS_MAX_RADIUS)
        return fail(OSBF_ERROR_UNSUPPORTED, "Gaussian radius %d above %d", r, OSBF_GAUSS_MAX_RADIUS);
    if (!(sigma > 0.0f)) return fail(OSBF_ERROR_INVALID_VALUE, "sigma must be > 0 (got %g)", (double)sigma);
    if (!src || !dst) return fail(OSBF_ERROR_INVALID_VALUE, "src and dst must be non-NULL");
    hipStream_t stream = (hipStream_t)stream_;
    const size_t n = (size_t)planes * H * W;
    const size_t bytes = n * sizeof(float);
    hipError_t e;
    if (T == 0 || r == 0) {
        if (src != dst && (e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
            return hip_fail(e, "copy");
        if (sel && T > 0 && (e = hipMemsetAsync(sel, OSBF_WIN_R, (size_t)T * n, stream)) != hipSuccess)
            return hip_fail(e, "memset sel");
        return OSBF_SUCCESS;
    }
    if ((T >= 2 || src == dst) && (!ws || ws_bytes < bytes))
        return fail(OSBF_ERROR_WORKSPACE, "workspace of %zu bytes required, got %zu", bytes, ws ? ws_bytes : 0);

    GaussLaunch a;
    a.planes = planes; a.H = H; a.W = W; a.r = r;
    if (!gauss_geometry(a)) return fail(OSBF_ERROR_INVALID_VALUE, "too many tiles");
    // taps g(u) = exp(-u^2 / (2 sigma^2)) (1 for sigma = infinity); the
    // normalisers come from the FP32 taps the kernel uses
    double zh = 0.0;
    for (int u = 0; u <= OSBF_GAUSS_MAX_R; ++u) {
        const double gu = std::isinf(sigma) ? 1.0 : std::exp(-(double)u * u / (2.0 * (double)sigma * sigma));
        a.g[u] = u <= r ? (float)gu : 0.0f;
        if (u <= r) zh += (double)a.g[u];
    }
    const double zf = 2.0 * zh - 1.0;
    a.w_q = (float)zf;
    a.w_h = (float)zh;
    a.N = (float)(zh * zh * zf);
    a.invN = (float)(1.0 / (zh * zh * zf));

    const float *cur = src;
    if (src == dst && (T % 2) == 1) {
        if ((e = hipMemcpyAsync(ws, src, bytes, hipMemcpyDeviceToDevice, stream)) != hipSuccess)
            return hip_fail(e, "copy to workspace");
        cur = (const float *)ws;
    }
    for (int t = 0; t < T; ++t) {
        float *out = ((T - 1 - t) % 2 == 0) ? dst : (float *)ws;
        a.src = cur;
        a.dst = out;
        a.sel = sel ? sel + (size_t)t * n : nullptr;
        if ((e = launch_gauss(a, stream)) != hipSuccess) return hip_fail(e, "Gaussian launch");
        cur = out;
    }
    return OSBF_SUCCESS;
}


osbf_status osbf_autotune(const void *src, void *dst, int32_t planes, int32_t H, int32_t W,
                          osbf_dtype dtype, int32_t r, int32_t T, void *stream_, int32_t *tile_w,
                          int32_t *tile_h, int32_t *fused) {
    g_last_error.clear();
    osbf_status st = check_sizes(planes, H, W, dtype, r, T);
    if (st != OSBF_SUCCESS) return st;
    if (!src || !dst || src == dst)
        return fail(OSBF_ERROR_INVALID_VALUE, "src and dst must be distinct non-NULL buffers");
    if (!tile_w || !tile_h || !fused) return fail(OSBF_ERROR_INVALID_VALUE, "output pointers must be non-NULL");
    *tile_w = *tile_h = *fused = 0;
    if (T == 0 || r == 0) return OSBF_SUCCESS;
    hipStream_t stream = (hipStream_t)stream_;
    const size_t limit = lds_limit();
    const int kmax = std::min(T, 6);
    // candidates: every fixed geometry and fusion depth that fits, and the
    // cost model's generic choice
    std::vector<Plan> cands;
    if (fixed_radius(r))
        for (int g = 1; g < NUM_GEOMS; ++g)
            for (int k = 1; k <= kmax; ++k) {
                const Plan p = make_plan(g, kGeomDims[g][0], kGeomDims[g][1], r, k);
                if (!p.tw || p.lds_bytes() > limit) continue;
                cands.push_back(p);
                if (stream_geom(g))  // and other rows per workgroup
                    for (int rows : {16, 32, 64, 96}) {
                        Plan q = p;
                        q.th = rows;
                        if (plan_rows(q, r) != plan_rows(p, r)) cands.push_back(q);
                    }
            }
    {
        Plan best;
        double best_cost = 1e300;
        for (int k = 1; k <= kmax; ++k)
            for (const auto &reg : kRegions) {
                const Plan p = make_plan(GEOM_GENERIC, reg[0], reg[1], r, k);
                if (!p.tw || p.lds_bytes() > limit) continue;
                const double c = plan_cost(p, H, W, r);
                if (c < best_cost) { best_cost = c; best = p; }
            }
        if (best.tw) cands.push_back(best);
    }
    if (cands.empty()) return fail(OSBF_ERROR_UNSUPPORTED, "radius %d does not fit the device's LDS", r);
    // the plan osbf_forward would use without tuning (the measured tables)
    size_t incumbent = cands.size();
    if (!getenv("OSBF_PLAN")) {
        const Plan t = choose_plan_model(planes, H, W, r, T, (int)dtype);
        for (size_t c = 0; c < cands.size() && incumbent == cands.size(); ++c)
            if (cands[c].geom == t.geom && cands[c].k == t.k && cands[c].tw == t.tw &&
                plan_rows(cands[c], r) == plan_rows(t, r))
                incumbent = c;
        if (incumbent == cands.size() && t.tw && t.lds_bytes() <= limit) cands.push_back(t);
    }
    // Every candidate gets its own event pair and a round is synchronised
    // once at its end, so the device runs the candidates back to back, as it
    // runs the sweeps of a call (a sync per candidate leaves it idle between
    // bursts and skews short measurements).  A warm-up burst first, then
    // kRounds rounds, each timing kReps launches of k sweeps per candidate after one
    // untimed launch; a candidate's figure is its best round.  Short bursts
    // still vary by several percent from run to run, so the plan the tables
    // would choose stays unless another beats it by more than 3%.
    constexpr int kReps = 8, kRounds = 3, kWarm = 8;
    const size_t nc = cands.size();
    std::vector<hipEvent_t> ev(2 * nc, nullptr);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < ev.size() && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    for (int i = 0; i < kWarm && e == hipSuccess; ++i)
        e = enqueue_forward(cands[0], cands[0].k, src, dst, nullptr, planes, H, W, r, dtype, stream);
    std::vector<double> per_sweep(nc, 1e300);
    for (int round = 0; round < kRounds && e == hipSuccess; ++round) {
        for (size_t c = 0; c < nc && e == hipSuccess; ++c) {
            const Plan &p = cands[c];
            e = enqueue_forward(p, p.k, src, dst, nullptr, planes, H, W, r, dtype, stream);
            if (e == hipSuccess) e = hipEventRecord(ev[2 * c], stream);
            for (int i = 0; i < kReps && e == hipSuccess; ++i)
                e = enqueue_forward(p, p.k, src, dst, nullptr, planes, H, W, r, dtype, stream);
            if (e == hipSuccess) e = hipEventRecord(ev[2 * c + 1], stream);
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[2 * nc - 1]);
        for (size_t c = 0; c < nc && e == hipSuccess; ++c) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[2 * c], ev[2 * c + 1]);
            if (e == hipSuccess) per_sweep[c] = std::min(per_sweep[c], (double)ms / (kReps * cands[c].k));
        }
    }
    for (hipEvent_t v : ev)
        if (v) (void)hipEventDestroy(v);
    if (e != hipSuccess) return hip_fail(e, "autotune launch");
    size_t pick = 0;
    for (size_t c = 1; c < nc; ++c)
        if (per_sweep[c] < per_sweep[pick]) pick = c;
    if (pick != incumbent && incumbent < nc && per_sweep[pick] > 0.97 * per_sweep[incumbent]) pick = incumbent;
    const Plan best = cands[pick];
    const std::string model = current_model();
    if (model.empty()) return fail(OSBF_ERROR_HIP, "device properties");
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        tune_file_read_locked();
        g_tune[std::make_tuple(model, r, (int)dtype, size_class(planes, H, W))] = best;
        tune_file_write_locked();
    }
    *tile_w = best.tw;
    *tile_h = plan_rows(best, r);
    *fused = best.k;
    return OSBF_SUCCESS;
}

void osbf_autotune_clear(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
    g_tune_batch.clear();
    g_tune_file_read = false;  // OSBF_TUNE_CACHE, if set, is read again on next use
}

}  // extern "C"
