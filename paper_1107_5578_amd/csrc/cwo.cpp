// Host runtime of libcwo: contexts, validation, tables, scratch and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <chrono>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <tuple>
#include <mutex>
#include <thread>
#include <vector>

#include "cwo.h"
#include "launch.hpp"

namespace {

constexpr int kMinN = 16;
constexpr int kMaxN = 4096;
constexpr size_t kFresnelCacheEntries = 8;

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

struct FresnelKey {
    int mx, nx, my, ny;
    double dx, dy, lam, z;
    bool unit;      // the shifted form's kernel factors: no constant, chirp pitches sqrt(p0 p1)
    bool analytic;  // the analytic transfer function instead of the DFT of the sampled chirps
    bool operator==(const FresnelKey& o) const {
        return mx == o.mx && nx == o.nx && my == o.my && ny == o.ny && dx == o.dx && dy == o.dy &&
               lam == o.lam && z == o.z && unit == o.unit && analytic == o.analytic;
    }
};

struct FresnelEntry {
    FresnelKey key;
    float2* h = nullptr;  // mx + my complex64: Hx (with C unless unit) then Hy
};

// A device buffer that only grows; growing waits for the device first because
// queued kernels on any stream may still use the old allocation.
struct Buffer {
    void* p = nullptr;
    size_t bytes = 0;
};

// Device memory one stream of work uses: the synchronous calls share the context's
// workspace; each serving slot has its own (so slots never touch each other's scratch or
// Fresnel factors, which are built on the slot's own stream).
struct Workspace {
    Buffer scratch;                   // padded planes
    Buffer fwork;                     // FP64 twiddles for the Fresnel factors
    Buffer ftab;                      // per-plane Fresnel factors of a z-stack chunk
    Buffer gsnum;                     // per-row error partials of the ping-pong iteration
    Buffer rwork;                     // range pre-pass of FP16 storage (scale, partials)
    Buffer fourier;                   // chirp tables of the Fresnel Fourier and shifted forms
    Buffer ework;                     // min/max partials of the scale epilogue
    Buffer pls;                       // FP64 point records of the point-light-source sums
    std::list<FresnelEntry> fresnel;  // most recently used first
    size_t budget = 0;                // 0: unbounded (serving slots are bounded by admission)
    // The one stream that uses this workspace (a serving slot's), or null when calls on
    // any stream may have used it: replacing a buffer first waits for that stream, or for
    // the whole device.
    hipStream_t owner = nullptr;
    // bytes of device memory held (buffers and Fresnel factors), readable from any thread
    std::atomic<size_t> total{0};
    size_t held() const { return total.load(); }
    hipError_t quiesce() const {
        return owner ? hipStreamSynchronize(owner) : hipDeviceSynchronize();
    }
    void release() {
        for (Buffer* b : {&scratch, &fwork, &ftab, &gsnum, &rwork, &fourier, &ework, &pls}) {
            if (b->p) (void)hipFree(b->p);
            b->p = nullptr;
            b->bytes = 0;
        }
        for (auto& e : fresnel) (void)hipFree(e.h);
        fresnel.clear();
        total = 0;
    }
};

struct Ticket {
    cwo_job job;
    int32_t state = 0;         // 0 queued, 1 running, 2 done, < 0 error status
    size_t footprint = 0;      // bytes reserved from admission to completion
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream (null: no ordering)
    double t_submit = 0, t_start = 0, t_done = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Workspace ws;
    std::vector<uint64_t> running;  // tickets of the batch in flight
};

}  // namespace

// Schedule picked by cwo_autotune for one parameter set (the distance does not change the
// work, so it is not part of the key; nz = 1 is the single-plane call).
struct TuneKey {
    int kind, nx, ny, precision, flags, nz;
    bool operator<(const TuneKey& o) const {
        return std::tie(kind, nx, ny, precision, flags, nz) <
               std::tie(o.kind, o.nx, o.ny, o.precision, o.flags, o.nz);
    }
};

// Serving slots per context (each its own stream and workspace).
constexpr int kSlots = 4;

struct cwo_ctx {
    int device = 0;
    size_t budget = 0;
    std::mutex mu;  // synchronous calls, twiddle tables, profiling
    cwo_status sticky = CWO_OK;
    std::map<int, float2*> twiddles;  // FP32 exp(-2 pi i k / M) per M
    std::atomic<size_t> twiddle_bytes{0};
    Workspace ws;                     // workspace of the synchronous calls
    // serving; lock order: qmu before mu
    std::mutex qmu;  // tickets, queue, admission state
    std::condition_variable qcv;
    std::map<uint64_t, Ticket> tickets;
    std::deque<uint64_t> queue;
    uint64_t next_ticket = 1;
    size_t reserved = 0;  // input and output bytes of admitted, unfinished requests
    Slot slots[kSlots];
    bool slots_ready = false;
    std::vector<hipEvent_t> ready_pool;  // spare events for submit-time ordering
    std::thread worker;
    bool stop = false;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    // serving batch limits (defaults, or the CWO_SERVE_* environment at creation)
    int serve_max_batch = 8;
    size_t serve_window = 256;
    size_t serve_batch_bytes = size_t(512) << 20;
    int serve_poll_us = 5;
    // per-kernel timing
    bool profiling = false;
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare;
    double prof_ms[CWO_STAGE_COUNT] = {};
    int64_t prof_n[CWO_STAGE_COUNT] = {};
    // schedules picked by cwo_autotune (the serving thread reads them too)
    std::mutex tmu;
    std::map<TuneKey, cwo_tuning> tuned;
};

namespace cwo {
thread_local StageTimer* g_stage_timer = nullptr;
}

namespace {

cwo_status dev_fail(cwo_ctx* c) {
    c->sticky = CWO_ERR_DEVICE;
    return CWO_ERR_DEVICE;
}

hipEvent_t take_event(cwo_ctx* c) {
    if (!c->spare.empty()) {
        hipEvent_t e = c->spare.back();
        c->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch through `fn` (returning hipError_t); with profiling on, the stage's kernels stamp
// a pair of events with their own start and end (a stage that launched nothing records
// nothing).
template <class F>
hipError_t timed(cwo_ctx* c, int stage, hipStream_t, F&& fn) {
    if (!c->profiling) return fn();
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return hipErrorOutOfMemory;
    cwo::StageTimer t{a, b, false};
    cwo::g_stage_timer = &t;
    const hipError_t e = fn();
    cwo::g_stage_timer = nullptr;
    if (t.started) {
        c->recs.push_back({stage, a, b});
    } else {
        c->spare.push_back(a);
        c->spare.push_back(b);
    }
    return e;
}

// Fold finished records into the totals (blocks until each stop event completes).
hipError_t drain_profile(cwo_ctx* c) {
    hipError_t err = hipSuccess;
    for (auto& r : c->recs) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e == hipSuccess) {
            c->prof_ms[r.stage] += ms;
            c->prof_n[r.stage] += 1;
        } else {
            err = e;
        }
        c->spare.push_back(r.a);
        c->spare.push_back(r.b);
    }
    c->recs.clear();
    return err;
}

#define CWO_HIP(ctx, call)                              \
    do {                                                \
        if ((call) != hipSuccess) return dev_fail(ctx); \
    } while (0)

const float2* twiddle_table(cwo_ctx* c, int m, hipStream_t s, cwo_status* st) {
    auto it = c->twiddles.find(m);
    if (it != c->twiddles.end()) return it->second;
    float2* tw = nullptr;
    if (hipMalloc(&tw, sizeof(float2) * (size_t)m) != hipSuccess) {
        *st = CWO_ERR_NOMEM;
        return nullptr;
    }
    // generated once on the caller's stream, then waited for, so later calls on any
    // stream see a complete table
    if (cwo::launch_twiddles(tw, m, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        (void)hipFree(tw);
        *st = dev_fail(c);
        return nullptr;
    }
    c->twiddles[m] = tw;
    c->twiddle_bytes += sizeof(float2) * (size_t)m;
    return tw;
}

// Grow b to at least `bytes` (contents are not kept). The old allocation may still be in
// use by queued kernels, so growing first waits for the workspace's stream (or device).
void* ensure(cwo_ctx* c, Workspace& ws, Buffer& b, size_t bytes, cwo_status* st) {
    if (b.bytes >= bytes) return b.p;
    if (ws.budget && ws.held() - b.bytes + bytes > ws.budget) {
        *st = CWO_ERR_NOMEM;
        return nullptr;
    }
    if (b.p) {
        if (ws.quiesce() != hipSuccess) {
            *st = dev_fail(c);
            return nullptr;
        }
        (void)hipFree(b.p);
        ws.total -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        b.p = nullptr;
        *st = CWO_ERR_NOMEM;
        return nullptr;
    }
    b.bytes = bytes;
    ws.total += bytes;
    return b.p;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Everything except the distance. low_prec: FP16/BF16 storage is built for this call
// (single padded propagations); elsewhere it is CWO_ERR_UNSUPPORTED.
cwo_status validate_geometry(const cwo_params* p, int kind, bool low_prec = false) {
    if (!p) return CWO_ERR_INVALID;
    if (kind != CWO_ANGULAR && kind != CWO_FRESNEL_CONV) return CWO_ERR_INVALID;
    if (p->kind != 0 && p->kind != kind) return CWO_ERR_INVALID;
    if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->wavelength)) return CWO_ERR_INVALID;
    const uint32_t allowed = CWO_FLAG_NOPAD | (kind == CWO_FRESNEL_CONV ? CWO_FLAG_FRESNEL_TF : 0u);
    if ((p->flags & ~allowed) != 0) return CWO_ERR_INVALID;
    if (p->precision < CWO_PREC_F32 || p->precision > CWO_PREC_BF16_STORAGE) return CWO_ERR_INVALID;
    if (!is_pow2(p->nx) || !is_pow2(p->ny) || p->nx < kMinN || p->ny < kMinN || p->nx > kMaxN ||
        p->ny > kMaxN)
        return CWO_ERR_UNSUPPORTED;
    if (p->precision != CWO_PREC_F32 && (!low_prec || (p->flags & CWO_FLAG_NOPAD)))
        return CWO_ERR_UNSUPPORTED;
    return CWO_OK;
}

cwo_status validate_z(double z, int kind) {
    if (!std::isfinite(z)) return CWO_ERR_INVALID;
    if (kind == CWO_FRESNEL_CONV && z == 0.0) return CWO_ERR_INVALID;
    return CWO_OK;
}

cwo_status validate(const cwo_params* p, int kind, bool low_prec = false) {
    cwo_status st = validate_geometry(p, kind, low_prec);
    if (st != CWO_OK) return st;
    return validate_z(p->z, kind);
}

struct Geometry {
    int nx, ny, mx, my;
};

Geometry geometry(const cwo_params* p) {
    const bool nopad = (p->flags & CWO_FLAG_NOPAD) != 0;
    return Geometry{p->nx, p->ny, nopad ? p->nx : 2 * p->nx, nopad ? p->ny : 2 * p->ny};
}

size_t elem_bytes(int precision) { return precision == CWO_PREC_F32 ? 8 : 4; }

int ilog2(int v) {
    int e = 0;
    while ((1 << (e + 1)) <= v) ++e;
    return e;
}

cwo::AsmScalars asm_scalars(const cwo_params* p, const Geometry& g, double z) {
    cwo::AsmScalars a;
    a.dfx = 1.0 / ((double)g.mx * p->dx);
    a.dfy = 1.0 / ((double)g.my * p->dy);
    a.lam = p->wavelength;
    a.zl = z / p->wavelength;
    return a;
}

// exp(i k z) / (i lambda z) * dx * dy, with k z reduced in revolutions in FP64
void fresnel_constant(double dx, double dy, double lam, double z, double* re, double* im) {
    const double t = z / lam;  // k z / (2 pi)
    const double r = t - std::nearbyint(t);
    const double ang = 2.0 * M_PI * r;
    const double amp = dx * dy / (lam * z);
    // (cos + i sin) / i = sin - i cos
    *re = amp * std::sin(ang);
    *im = -amp * std::cos(ang);
}

// exp(i k z), k z reduced in revolutions in FP64 (constant of the analytic transfer function)
void phase_constant(double lam, double z, double* re, double* im) {
    const double t = z / lam;
    const double ang = 2.0 * M_PI * (t - std::nearbyint(t));
    *re = std::cos(ang);
    *im = std::sin(ang);
}

cwo::FresnelPlanes fresnel_planes(const cwo_params* p, const Geometry& g, const double* z, int nz) {
    cwo::FresnelPlanes fp;
    std::memset(&fp, 0, sizeof(fp));
    fp.mx = g.mx;
    fp.nx = g.nx;
    fp.my = g.my;
    fp.ny = g.ny;
    fp.dx = p->dx;
    fp.dy = p->dy;
    fp.nz = nz;
    fp.analytic = (p->flags & CWO_FLAG_FRESNEL_TF) != 0;
    for (int k = 0; k < nz; ++k) {
        fp.inv2lz[k] = 0.5 / (p->wavelength * z[k]);
        fp.hlz[k] = 0.5 * p->wavelength * z[k];
        if (fp.analytic)
            phase_constant(p->wavelength, z[k], &fp.cre[k], &fp.cim[k]);
        else
            fresnel_constant(p->dx, p->dy, p->wavelength, z[k], &fp.cre[k], &fp.cim[k]);
    }
    return fp;
}

// Fresnel factors of one plane, cached per parameter set.
// Transformed 1-D chirps of the Fresnel kernel, cached per parameter set (most recently
// used first). unit: the shifted form's kernel (chirp pitch sqrt(p0 p1) passed as
// dx, dy, no constant).
const float2* factor_table(cwo_ctx* c, Workspace& ws, const FresnelKey& key, hipStream_t s,
                           cwo_status* st) {
    for (auto it = ws.fresnel.begin(); it != ws.fresnel.end(); ++it) {
        if (it->key == key) {
            ws.fresnel.splice(ws.fresnel.begin(), ws.fresnel, it);
            return ws.fresnel.front().h;
        }
    }
    const size_t len = (size_t)(key.mx + key.my);
    double2* work = (double2*)ensure(c, ws, ws.fwork, sizeof(double2) * len, st);
    if (!work) return nullptr;
    if (ws.fresnel.size() >= kFresnelCacheEntries) {
        FresnelEntry old = ws.fresnel.back();
        ws.fresnel.pop_back();
        if (ws.quiesce() != hipSuccess) {
            *st = dev_fail(c);
            return nullptr;
        }
        (void)hipFree(old.h);
        ws.total -= sizeof(float2) * (size_t)(old.key.mx + old.key.my);
    }
    FresnelEntry e;
    e.key = key;
    if (hipMalloc(&e.h, sizeof(float2) * len) != hipSuccess) {
        *st = CWO_ERR_NOMEM;
        return nullptr;
    }
    ws.total += sizeof(float2) * len;
    cwo::FresnelPlanes fp;
    std::memset(&fp, 0, sizeof(fp));
    fp.mx = key.mx;
    fp.nx = key.nx;
    fp.my = key.my;
    fp.ny = key.ny;
    fp.dx = key.dx;
    fp.dy = key.dy;
    fp.nz = 1;
    fp.inv2lz[0] = 0.5 / (key.lam * key.z);
    fp.hlz[0] = 0.5 * key.lam * key.z;
    fp.analytic = key.analytic;
    if (key.unit) {
        fp.cre[0] = 1.0;
        fp.cim[0] = 0.0;
    } else if (key.analytic) {
        phase_constant(key.lam, key.z, &fp.cre[0], &fp.cim[0]);
    } else {
        fresnel_constant(key.dx, key.dy, key.lam, key.z, &fp.cre[0], &fp.cim[0]);
    }
    if (timed(c, CWO_STAGE_TABLES, s, [&] { return cwo::launch_fresnel_planes(work, e.h, fp, s); }) !=
        hipSuccess) {
        (void)hipFree(e.h);
        ws.total -= sizeof(float2) * len;
        *st = dev_fail(c);
        return nullptr;
    }
    ws.fresnel.push_front(e);
    return e.h;
}

const float2* fresnel_factors(cwo_ctx* c, Workspace& ws, const cwo_params* p, const Geometry& g,
                              hipStream_t s, cwo_status* st) {
    const FresnelKey key{g.mx, g.nx, g.my, g.ny, p->dx, p->dy, p->wavelength, p->z, false,
                         (p->flags & CWO_FLAG_FRESNEL_TF) != 0};
    return factor_table(c, ws, key, s, st);
}

TuneKey tune_key(const cwo_params* p, int kind, int nz) {
    return TuneKey{kind, p->nx, p->ny, p->precision, (int)p->flags, nz};
}

// The tuned schedule of a parameter set (all zero: none, the defaults apply).
cwo_tuning tuned_for(cwo_ctx* c, const cwo_params* p, int kind, int nz) {
    std::lock_guard<std::mutex> g(c->tmu);
    auto it = c->tuned.find(tune_key(p, kind, nz));
    return it == c->tuned.end() ? cwo_tuning{0, 0, 0.0f, 0, 0} : it->second;
}

// Whether the tiled plane can be used for this geometry at all (padded planes of
// 2048 <= Mx <= 8192, as the default rule).
bool tiles_possible(const Geometry& g) {
    return g.mx == 2 * g.nx && g.my == 2 * g.ny && g.mx >= 2048 && g.mx <= 8192;
}

// Plane layout of a single propagation: the tuned one if any (1 row-major, 2 tiled), else
// the default rule.
int plane_layout(const Geometry& g, const cwo_tuning& t) {
    if (t.layout == 1) return 0;
    if (t.layout == 2 && tiles_possible(g)) return 1;
    return cwo::tiled_ok(g.nx, g.ny, g.mx, g.my) ? 1 : 0;
}

// Column forms of a plane laid out as `layout` (1 tiled): both forms for padded columns of
// 4096 or 8192 on the tiled plane, else only the default.
bool col_forms_possible(const Geometry& g, int layout) {
    return layout == 1 && g.my == 2 * g.ny && (g.my == 4096 || g.my == 8192);
}

void set_tuned(cwo_ctx* c, const TuneKey& k, const cwo_tuning* t) {
    std::lock_guard<std::mutex> g(c->tmu);
    if (t) c->tuned[k] = *t;
    else c->tuned.erase(k);
}

// ---- tune cache ----------------------------------------------------------------------
//
// With CWO_TUNE_CACHE naming a file, cwo_create reads the schedules stored there and every
// successful cwo_autotune rewrites the file with all schedules the context knows: a JSON
// array of flat objects, one per line, e.g.
//   {"kind": 1, "nx": 2048, "ny": 2048, "precision": 0, "flags": 0, "nz": 1,
//    "row_form": 1, "zchunk": 0, "layout": 2, "us_per_plane": 126.5, "col_form": 1}
// (written on one line). Lines that do not parse are ignored; a missing file is no error.
const char* tune_cache_path() {
    const char* p = std::getenv("CWO_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

void load_tune_cache(cwo_ctx* c) {
    const char* path = tune_cache_path();
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        TuneKey k{};
        cwo_tuning t{};
        const int n = std::sscanf(line,
                                  " {\"kind\": %d, \"nx\": %d, \"ny\": %d, \"precision\": %d, "
                                  "\"flags\": %d, \"nz\": %d, \"row_form\": %d, \"zchunk\": %d, "
                                  "\"layout\": %d, \"us_per_plane\": %f, \"col_form\": %d",
                                  &k.kind, &k.nx, &k.ny, &k.precision, &k.flags, &k.nz, &t.row_form,
                                  &t.zchunk, &t.layout, &t.us_per_plane, &t.col_form);
        // (records written before the column form existed end after us_per_plane)
        if (n >= 10) set_tuned(c, k, &t);
    }
    std::fclose(f);
}

void save_tune_cache(cwo_ctx* c) {
    const char* path = tune_cache_path();
    if (!path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::lock_guard<std::mutex> g(c->tmu);
    std::fprintf(f, "[\n");
    size_t i = 0;
    for (const auto& kv : c->tuned) {
        const TuneKey& k = kv.first;
        const cwo_tuning& t = kv.second;
        std::fprintf(f,
                     " {\"kind\": %d, \"nx\": %d, \"ny\": %d, \"precision\": %d, \"flags\": %d, "
                     "\"nz\": %d, \"row_form\": %d, \"zchunk\": %d, \"layout\": %d, "
                     "\"us_per_plane\": %.3f, \"col_form\": %d}%s\n",
                     k.kind, k.nx, k.ny, k.precision, k.flags, k.nz, t.row_form, t.zchunk, t.layout,
                     (double)t.us_per_plane, t.col_form, ++i < c->tuned.size() ? "," : "");
    }
    std::fprintf(f, "]\n");
    const bool ok = std::fclose(f) == 0;
    if (ok) std::rename(tmp.c_str(), path);
    else std::remove(tmp.c_str());
}

cwo_status begin(cwo_ctx* c) {
    if (c->sticky != CWO_OK) return c->sticky;
    if (hipSetDevice(c->device) != hipSuccess) return dev_fail(c);
    return CWO_OK;
}

// intensity: out is float [ny][nx] and receives |u|^2 of the result (stored by the row
// inverse pass instead of u).
cwo_status propagate_locked(cwo_ctx* c, Workspace& ws, const cwo_params* p, int kind,
                            const void* in, void* out, hipStream_t s,
                            const cwo::AsmShift* shift = nullptr, bool intensity = false) {
    cwo_status st = CWO_OK;
    const Geometry g = geometry(p);
    const float2* twx = twiddle_table(c, g.mx, s, &st);
    if (!twx) return st;
    const float2* twy = twiddle_table(c, g.my, s, &st);
    if (!twy) return st;
    void* buf = ensure(c, ws, ws.scratch, elem_bytes(p->precision) * (size_t)g.ny * g.mx, &st);
    if (!buf) return st;
    const float2* fin = (const float2*)in;
    float2* fout = (float2*)out;
    const float2* h = nullptr;
    if (kind == CWO_FRESNEL_CONV) {
        h = fresnel_factors(c, ws, p, g, s, &st);
        if (!h) return st;
    }
    cwo::Storage sto;  // complex64: no intermediate scaling, 1/(Mx My) at the end
    sto.out_scale = 1.0f / ((float)g.mx * (float)g.my);  // power of two: exact
    const cwo_tuning tune = tuned_for(c, p, kind, 1);
    sto.row_form = tune.row_form;
    sto.layout = plane_layout(g, tune);
    sto.col_form = col_forms_possible(g, sto.layout) && tune.col_form >= 0 && tune.col_form <= 2
                       ? tune.col_form
                       : 0;
    if (p->precision != CWO_PREC_F32) {
        // FP16/BF16 storage: 2^-floor(log2(Mx)/2) before the row transform, 1/My in the
        // column pass, the rest of 1/Mx at the end (all powers of two); FP16 also scales
        // the field by 2^-e, e the exponent of its largest component, found on the device
        sto.prec = p->precision == CWO_PREC_F16_STORAGE ? 1 : 2;
        const int kx = ilog2(g.mx) / 2;
        sto.in_scale = std::ldexp(1.0f, -kx);
        sto.col_scale = 1.0f / (float)g.my;
        sto.out_scale = std::ldexp(1.0f, kx) / (float)g.mx;
        if (sto.prec == 1) {
            float* rw = (float*)ensure(c, ws, ws.rwork, sizeof(float) * (2 + cwo::kRangeBlocks), &st);
            if (!rw) return st;
            CWO_HIP(c, cwo::launch_range_scale(fin, (size_t)g.ny * g.nx, rw, s));
            sto.dyn_scale = rw;
            sto.dyn_inv = rw + 1;
        }
    }
    CWO_HIP(c, timed(c, CWO_STAGE_ROW_FWD, s, [&] {
                return cwo::launch_row_fwd(fin, buf, g.nx, g.ny, g.mx, 1, 0, 0, sto, twx, s);
            }));
    if (kind == CWO_ANGULAR && shift) {
        const cwo::AsmScalars a = asm_scalars(p, g, p->z);
        float* masks = (float*)ensure(c, ws, ws.fourier, sizeof(float) * (size_t)(g.mx + g.my), &st);
        if (!masks) return st;
        CWO_HIP(c, timed(c, CWO_STAGE_COL, s, [&] {
                    return cwo::launch_col_asm_shifted(buf, g.ny, g.my, g.mx, a, *shift, masks,
                                                       sto, twy, s);
                }));
    } else if (kind == CWO_ANGULAR) {
        const cwo::AsmScalars a = asm_scalars(p, g, p->z);
        CWO_HIP(c, timed(c, CWO_STAGE_COL, s, [&] {
                    return cwo::launch_col_asm(buf, g.ny, g.my, g.mx, 1, 0, a, sto, twy, s);
                }));
    } else {
        CWO_HIP(c, timed(c, CWO_STAGE_COL, s, [&] {
                    return cwo::launch_col_fresnel(buf, g.ny, g.my, g.mx, 1, 0, h, h + g.mx, sto, twy,
                                                   s);
                }));
    }
    CWO_HIP(c, timed(c, CWO_STAGE_ROW_INV, s, [&] {
                if (intensity)
                    return cwo::launch_row_inv_intensity(buf, (float*)out, g.nx, g.ny, g.mx, sto,
                                                         twx, s);
                return cwo::launch_row_inv(buf, fout, g.nx, g.ny, g.mx, 1, 0, 0, sto, twx, s);
            }));
    return CWO_OK;
}

cwo_status propagate(cwo_ctx* c, const cwo_params* p, int kind, const void* in, void* out,
                     void* stream, const cwo::AsmShift* shift = nullptr,
                     bool intensity = false) {
    if (!c) return CWO_ERR_INVALID;
    cwo_status st = validate(p, kind, true);
    if (st != CWO_OK) return st;
    if (!in || !out) return CWO_ERR_INVALID;
    std::lock_guard<std::mutex> lock(c->mu);
    st = begin(c);
    if (st != CWO_OK) return st;
    return propagate_locked(c, c->ws, p, kind, in, out, (hipStream_t)stream, shift, intensity);
}

// One field to nz distances; plane k goes to outs[k]. The row transform of the field
// and the forward column transforms run once; planes are processed in chunks of at
// most kZChunk that fit the scratch budget.
cwo_status zstack_locked(cwo_ctx* c, Workspace& ws, const cwo_params* p, int kind, const double* z,
                         int nz, const void* in, void* const* outs, hipStream_t s) {
    cwo_status st = CWO_OK;
    const Geometry g = geometry(p);
    const float2* twx = twiddle_table(c, g.mx, s, &st);
    if (!twx) return st;
    const float2* twy = twiddle_table(c, g.my, s, &st);
    if (!twy) return st;
    const size_t plane = (size_t)g.ny * g.mx;
    const size_t len = (size_t)(g.mx + g.my);
    const size_t eb = elem_bytes(p->precision);  // bytes per stored complex value
    // chunk size: the shared spectrum and all planes of a chunk within the budget
    int zc = std::min(nz, cwo::kZChunk);
    const cwo_tuning tune = tuned_for(c, p, kind, nz);
    if (tune.zchunk > 0) zc = std::min(zc, tune.zchunk);
    if (ws.budget) {
        const size_t fres = kind == CWO_FRESNEL_CONV ? sizeof(float2) * len : 0;
        const size_t per_plane = eb * plane + fres;
        const size_t base = eb * plane + (kind == CWO_FRESNEL_CONV ? sizeof(double2) * len : 0);
        if (ws.budget < base + per_plane) return CWO_ERR_NOMEM;
        const size_t fit = (ws.budget - base) / per_plane;
        zc = (int)std::min<size_t>((size_t)zc, fit);
    }
    char* buf = (char*)ensure(c, ws, ws.scratch, eb * plane * (size_t)(1 + zc), &st);
    if (!buf) return st;
    void* spec = buf;
    void* zbuf = buf + eb * plane;
    float2* tabs = nullptr;
    double2* work = nullptr;
    if (kind == CWO_FRESNEL_CONV) {
        tabs = (float2*)ensure(c, ws, ws.ftab, sizeof(float2) * len * zc, &st);
        if (!tabs) return st;
        work = (double2*)ensure(c, ws, ws.fwork, sizeof(double2) * len, &st);
        if (!work) return st;
    }
    // storage of the shared spectrum and the planes: complex64 with 1/(Mx My) at the end,
    // or 16-bit pairs with the power-of-two scalings of a single propagation
    cwo::Storage sto;
    sto.out_scale = 1.0f / ((float)g.mx * (float)g.my);
    sto.row_form = tune.row_form;
    if (p->precision != CWO_PREC_F32) {
        sto.prec = p->precision == CWO_PREC_F16_STORAGE ? 1 : 2;
        const int kx = ilog2(g.mx) / 2;
        sto.in_scale = std::ldexp(1.0f, -kx);
        sto.col_scale = 1.0f / (float)g.my;
        sto.out_scale = std::ldexp(1.0f, kx) / (float)g.mx;
        if (sto.prec == 1) {
            float* rw = (float*)ensure(c, ws, ws.rwork, sizeof(float) * (2 + cwo::kRangeBlocks), &st);
            if (!rw) return st;
            CWO_HIP(c, cwo::launch_range_scale((const float2*)in, (size_t)g.ny * g.nx, rw, s));
            sto.dyn_scale = rw;
            sto.dyn_inv = rw + 1;
        }
    }
    CWO_HIP(c, timed(c, CWO_STAGE_ROW_FWD, s, [&] {
                return cwo::launch_row_fwd((const float2*)in, spec, g.nx, g.ny, g.mx, 1, 0, 0, sto,
                                           twx, s);
            }));
    for (int k0 = 0; k0 < nz; k0 += zc) {
        const int n = std::min(zc, nz - k0);
        cwo::ZChunk ch;
        std::memset(&ch, 0, sizeof(ch));
        ch.nz = n;
        for (int k = 0; k < n; ++k) {
            ch.zl[k] = z[k0 + k] / p->wavelength;
            ch.out[k] = (float2*)outs[k0 + k];
        }
        if (kind == CWO_ANGULAR) {
            const cwo::AsmScalars a = asm_scalars(p, g, 0.0);
            CWO_HIP(c, timed(c, CWO_STAGE_COL_Z, s, [&] {
                        return cwo::launch_col_z_asm(spec, zbuf, g.ny, g.my, g.mx, plane, a, ch, sto,
                                                     twy, s);
                    }));
        } else {
            const cwo::FresnelPlanes fp = fresnel_planes(p, g, z + k0, n);
            CWO_HIP(c, timed(c, CWO_STAGE_TABLES, s,
                             [&] { return cwo::launch_fresnel_planes(work, tabs, fp, s); }));
            CWO_HIP(c, timed(c, CWO_STAGE_COL_Z, s, [&] {
                        return cwo::launch_col_z_fresnel(spec, zbuf, g.ny, g.my, g.mx, plane, tabs, n,
                                                         sto, twy, s);
                    }));
        }
        CWO_HIP(c, timed(c, CWO_STAGE_ROW_INV, s, [&] {
                    return cwo::launch_row_inv_z(zbuf, ch, g.nx, g.ny, g.mx, plane, sto, twx, s);
                }));
    }
    return CWO_OK;
}

// Jobs that run as one z-stack: the same field and geometry, complex64 storage (z-stacks
// keep complex64 planes; 16-bit requests run singly).
bool same_group(const cwo_job& a, const cwo_job& b) {
    return a.in == b.in && a.p.nx == b.p.nx && a.p.ny == b.p.ny && a.p.dx == b.p.dx &&
           a.p.dy == b.p.dy && a.p.wavelength == b.p.wavelength && a.p.kind == b.p.kind &&
           a.p.precision == CWO_PREC_F32 && b.p.precision == CWO_PREC_F32 &&
           a.p.flags == b.p.flags;
}

cwo_status validate_jobs(const cwo_job* jobs, int njobs) {
    for (int i = 0; i < njobs; ++i) {
        const bool grouped = (i > 0 && same_group(jobs[i - 1], jobs[i])) ||
                             (i + 1 < njobs && same_group(jobs[i], jobs[i + 1]));
        cwo_status st = validate(&jobs[i].p, jobs[i].p.kind, !grouped);
        if (st != CWO_OK) return st;
        if (!jobs[i].in || !jobs[i].out) return CWO_ERR_INVALID;
    }
    return CWO_OK;
}

// A job that can run as one plane of a mixed batch: complex64 storage, and for ASM a
// transfer function in the fast form (the exact form runs singly).
bool batchable(const cwo_job& j) {
    if (j.p.precision != CWO_PREC_F32) return false;
    if (j.p.kind == CWO_FRESNEL_CONV) return true;
    if (j.p.kind != CWO_ANGULAR) return false;
    const Geometry g = geometry(&j.p);
    return cwo::asm_plane_tf(asm_scalars(&j.p, g, j.p.z), g.mx, g.my).form <= 1;
}

// Consecutive jobs on the same field and geometry run as one z-stack; the rest singly.
// Jobs of one geometry (sizes, pitch, flags) on different fields run as one batch per pass,
// each plane with its own distance, wavelength and kind.
bool same_params(const cwo_job& a, const cwo_job& b) {
    return a.p.nx == b.p.nx && a.p.ny == b.p.ny && a.p.dx == b.p.dx && a.p.dy == b.p.dy &&
           a.p.flags == b.p.flags && batchable(a) && batchable(b);
}

// Jobs [i, j) of one geometry, one batch per pass, in chunks of at most kZChunk planes
// that fit the budget. Each plane gets the transfer function its single call would use:
// the ASM fast form for its scalars, or Fresnel factors computed for the chunk's Fresnel
// planes (the same kernel and arithmetic as the cached single-call factors). Every field
// is read by the first pass before the last pass writes any output, so a batch must not
// read another batch member's output.
cwo_status batch_locked(cwo_ctx* c, Workspace& ws, const cwo_job* jobs, int n, hipStream_t s) {
    cwo_status st = CWO_OK;
    const cwo_params* p = &jobs[0].p;
    const Geometry g = geometry(p);
    const float2* twx = twiddle_table(c, g.mx, s, &st);
    if (!twx) return st;
    const float2* twy = twiddle_table(c, g.my, s, &st);
    if (!twy) return st;
    const size_t plane = (size_t)g.ny * g.mx;
    const size_t len = (size_t)(g.mx + g.my);
    int nfres = 0;
    for (int k = 0; k < n; ++k) nfres += jobs[k].p.kind == CWO_FRESNEL_CONV;
    int chunk = std::min(n, cwo::kZChunk);
    if (ws.budget) {
        const size_t other = ws.held() - ws.scratch.bytes - ws.ftab.bytes - ws.fwork.bytes;
        const size_t fixed = nfres ? sizeof(double2) * len : 0;
        const size_t per = sizeof(float2) * plane + (nfres ? sizeof(float2) * len : 0);
        const size_t fit = ws.budget > other + fixed ? (ws.budget - other - fixed) / per : 0;
        if (fit == 0) return CWO_ERR_NOMEM;
        chunk = (int)std::min<size_t>((size_t)chunk, fit);
    }
    float2* buf = (float2*)ensure(c, ws, ws.scratch, sizeof(float2) * plane * (size_t)chunk, &st);
    if (!buf) return st;
    float2* ftab = nullptr;
    double2* work = nullptr;
    if (nfres) {
        ftab = (float2*)ensure(c, ws, ws.ftab, sizeof(float2) * len * (size_t)std::min(chunk, nfres), &st);
        if (!ftab) return st;
        work = (double2*)ensure(c, ws, ws.fwork, sizeof(double2) * len, &st);
        if (!work) return st;
    }
    const float scale = 1.0f / ((float)g.mx * (float)g.my);
    const int layout = cwo::tiled_ok(g.nx, g.ny, g.mx, g.my) ? 1 : 0;
    const bool analytic = (p->flags & CWO_FLAG_FRESNEL_TF) != 0;
    for (int k0 = 0; k0 < n; k0 += chunk) {
        const int nb = std::min(chunk, n - k0);
        cwo::InTable ins;
        cwo::OutTable outs;
        cwo::PlaneTF tab[cwo::kZChunk];
        std::memset(tab, 0, sizeof(tab));
        cwo::FresnelPlanes fp;
        std::memset(&fp, 0, sizeof(fp));
        fp.mx = g.mx;
        fp.nx = g.nx;
        fp.my = g.my;
        fp.ny = g.ny;
        fp.dx = p->dx;
        fp.dy = p->dy;
        fp.analytic = analytic;
        for (int k = 0; k < cwo::kZChunk; ++k) {
            ins.in[k] = k < nb ? (const float2*)jobs[k0 + k].in : nullptr;
            outs.out[k] = k < nb ? (float2*)jobs[k0 + k].out : nullptr;
        }
        for (int k = 0; k < nb; ++k) {
            const cwo_params* q = &jobs[k0 + k].p;
            if (q->kind == CWO_ANGULAR) {
                tab[k] = cwo::asm_plane_tf(asm_scalars(q, g, q->z), g.mx, g.my);
            } else {
                const int f = fp.nz++;
                fp.inv2lz[f] = 0.5 / (q->wavelength * q->z);
                fp.hlz[f] = 0.5 * q->wavelength * q->z;
                if (analytic)
                    phase_constant(q->wavelength, q->z, &fp.cre[f], &fp.cim[f]);
                else
                    fresnel_constant(q->dx, q->dy, q->wavelength, q->z, &fp.cre[f], &fp.cim[f]);
                tab[k].form = 3;
                tab[k].h = ftab + (size_t)f * len;
            }
        }
        if (fp.nz > 0)
            CWO_HIP(c, timed(c, CWO_STAGE_TABLES, s,
                             [&] { return cwo::launch_fresnel_planes(work, ftab, fp, s); }));
        CWO_HIP(c, timed(c, CWO_STAGE_ROW_FWD, s, [&] {
                    return cwo::launch_row_fwd_tab(ins, buf, g.nx, g.ny, g.mx, nb, plane, twx, s,
                                                   layout);
                }));
        // one column launch per transfer-function form present
        bool present[4] = {false, false, false, false};
        for (int k = 0; k < nb; ++k) present[tab[k].form] = true;
        for (int form : {0, 1, 3}) {
            if (!present[form]) continue;
            CWO_HIP(c, timed(c, CWO_STAGE_COL, s, [&] {
                        return cwo::launch_col_mixed(buf, g.ny, g.my, g.mx, nb, plane, tab, form,
                                                     twy, s, layout);
                    }));
        }
        CWO_HIP(c, timed(c, CWO_STAGE_ROW_INV, s, [&] {
                    return cwo::launch_row_inv_tab(buf, outs, g.nx, g.ny, g.mx, nb, plane, scale,
                                                   twx, s, layout);
                }));
    }
    return CWO_OK;
}

// Length of the run of jobs from i of one geometry (same_params) whose inputs are all
// different and none of which reads another member's output.
int batch_run(const cwo_job* jobs, int i, int njobs) {
    int j = i + 1;
    while (j < njobs && j - i < cwo::kZChunk && same_params(jobs[i], jobs[j])) {
        bool ok = true;
        for (int k = i; k < j && ok; ++k)
            ok = jobs[k].in != jobs[j].in && jobs[k].out != jobs[j].in && jobs[k].in != jobs[j].out &&
                 jobs[k].out != jobs[j].out;
        if (!ok) break;
        ++j;
    }
    return j - i;
}

// How run_jobs groups a job list: consecutive jobs on one field with one geometry form a
// z-stack; runs of one geometry on distinct fields a batch; the rest run singly.
struct Group {
    enum Type { SINGLE, ZSTACK, BATCH } type;
    int i, j;  // jobs [i, j)
};

std::vector<Group> plan_groups(const cwo_job* jobs, int njobs) {
    std::vector<Group> gs;
    int i = 0;
    while (i < njobs) {
        int j = i + 1;
        while (j < njobs && same_group(jobs[i], jobs[j])) ++j;
        if (j - i == 1 && batch_run(jobs, i, njobs) > 1)
            gs.push_back({Group::BATCH, i, i + batch_run(jobs, i, njobs)});
        else
            gs.push_back({j - i == 1 ? Group::SINGLE : Group::ZSTACK, i, j});
        i = gs.back().j;
    }
    return gs;
}

cwo_status run_jobs(cwo_ctx* c, Workspace& ws, const cwo_job* jobs, int njobs, hipStream_t s) {
    for (const Group& gr : plan_groups(jobs, njobs)) {
        cwo_status st = CWO_OK;
        const int i = gr.i, n = gr.j - gr.i;
        if (gr.type == Group::BATCH) {
            st = batch_locked(c, ws, jobs + i, n, s);
        } else if (gr.type == Group::SINGLE) {
            st = propagate_locked(c, ws, &jobs[i].p, jobs[i].p.kind, jobs[i].in, jobs[i].out, s);
        } else {
            std::vector<double> z;
            std::vector<void*> outs;
            for (int k = gr.i; k < gr.j; ++k) {
                z.push_back(jobs[k].p.z);
                outs.push_back(jobs[k].out);
            }
            st = zstack_locked(c, ws, &jobs[i].p, jobs[i].p.kind, z.data(), n, jobs[i].in,
                               outs.data(), s);
        }
        if (st != CWO_OK) return st;
    }
    return CWO_OK;
}

// Largest size of each workspace buffer a job list needs on an unbounded workspace (the
// serving slots'), and how many Fresnel factor entries it may add.
struct WsNeed {
    size_t scratch = 0, fwork = 0, ftab = 0, rwork = 0, factors = 0;
};

WsNeed jobs_need(cwo_ctx* c, const cwo_job* jobs, int njobs) {
    WsNeed w;
    for (const Group& gr : plan_groups(jobs, njobs)) {
        const cwo_params* p = &jobs[gr.i].p;
        const Geometry g = geometry(p);
        const size_t plane = (size_t)g.ny * g.mx;
        const size_t len = (size_t)(g.mx + g.my);
        const bool fres = p->kind == CWO_FRESNEL_CONV;
        const int n = gr.j - gr.i;
        if (gr.type == Group::ZSTACK) {
            int zc = std::min(n, cwo::kZChunk);
            const cwo_tuning t = tuned_for(c, p, p->kind, n);
            if (t.zchunk > 0) zc = std::min(zc, t.zchunk);
            w.scratch = std::max(w.scratch, sizeof(float2) * plane * (size_t)(1 + zc));
            if (fres) {
                w.ftab = std::max(w.ftab, sizeof(float2) * len * (size_t)zc);
                w.fwork = std::max(w.fwork, sizeof(double2) * len);
            }
        } else if (gr.type == Group::BATCH) {
            const int nb = std::min(n, cwo::kZChunk);
            int nf = 0;
            for (int k = gr.i; k < gr.j; ++k) nf += jobs[k].p.kind == CWO_FRESNEL_CONV;
            w.scratch = std::max(w.scratch, sizeof(float2) * plane * (size_t)nb);
            if (nf) {
                w.ftab = std::max(w.ftab, sizeof(float2) * len * (size_t)std::min(nf, nb));
                w.fwork = std::max(w.fwork, sizeof(double2) * len);
            }
        } else {
            w.scratch = std::max(w.scratch, elem_bytes(p->precision) * plane);
            if (p->precision == CWO_PREC_F16_STORAGE)
                w.rwork = std::max(w.rwork, sizeof(float) * (2 + cwo::kRangeBlocks));
            if (fres) {
                w.fwork = std::max(w.fwork, sizeof(double2) * len);
                w.factors += sizeof(float2) * len;
            }
        }
    }
    return w;
}

// Bytes workspace ws would add to hold what `need` asks for (its cache may also evict).
size_t growth(const Workspace& ws, const WsNeed& need) {
    auto more = [](size_t have, size_t want) { return want > have ? want - have : 0; };
    return more(ws.scratch.bytes, need.scratch) + more(ws.fwork.bytes, need.fwork) +
           more(ws.ftab.bytes, need.ftab) + more(ws.rwork.bytes, need.rwork) + need.factors;
}

// ---- serving: continuous batching ------------------------------------------------
//
// A scheduler thread per context admits queued requests in arrival order when a slot
// (its own HIP stream, workspace and completion event) is free and the request fits the
// HBM budget: the input and output fields of every admitted, unfinished request, the
// memory every workspace of the context holds, and what the new batch would add to its
// slot's workspace, together at most the budget. Idle slots give their workspaces back
// when memory is short. A free slot takes the head request and, from the first
// serve_window queued requests in arrival order, those of the head's geometry (sizes, pitch,
// flags, precision) that fit, up to serve_max_batch requests and serve_batch_bytes of padded
// planes, as one batch run on its stream: one launch per pass for the whole batch, a z-stack for requests
// on one field. Queued requests do not depend on each other (an input is complete when it
// is submitted), but a request that shares a buffer with an earlier one left in the queue
// is not taken ahead of it. Every request becomes the head in arrival order, so none waits
// behind later ones for long. Slots run concurrently, so work from different arrivals
// overlaps on the device. Launching happens outside the queue lock, so submit and poll
// never wait for kernel launches or allocations.

// (the limits are the context's serve_* fields: by default 8 requests, a window of 256 and
// 512 MiB of padded planes, with a 5 us polling interval while slots run, or
// CWO_SERVE_MAX_BATCH, CWO_SERVE_WINDOW, CWO_SERVE_BATCH_MIB and CWO_SERVE_POLL_US from the
// environment when the context is created. On the 10k-request mix of four sizes, 512 MiB
// against 1 GiB kept the throughput and cut the p99 latency at 0.95 load from 22 to 13 ms;
// 2 GiB let batches of 4096^2 requests hold the memory other slots need: 1.03x plain
// instead of 1.2x; 256 MiB split the 2048^2 batches: 1.14x.)
void read_serve_env(cwo_ctx* c) {
    auto get = [](const char* name, long lo, long hi, long dflt) {
        const char* v = std::getenv(name);
        if (!v || !*v) return dflt;
        char* end = nullptr;
        const long x = std::strtol(v, &end, 10);
        return (end && *end == 0 && x >= lo && x <= hi) ? x : dflt;
    };
    c->serve_max_batch = (int)get("CWO_SERVE_MAX_BATCH", 1, cwo::kZChunk, c->serve_max_batch);
    c->serve_window = (size_t)get("CWO_SERVE_WINDOW", 1, 4096, (long)c->serve_window);
    c->serve_batch_bytes =
        (size_t)get("CWO_SERVE_BATCH_MIB", 1, 1 << 20, (long)(c->serve_batch_bytes >> 20)) << 20;
    c->serve_poll_us = (int)get("CWO_SERVE_POLL_US", 1, 10000, c->serve_poll_us);
}

double now_s(const cwo_ctx* c) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - c->t0).count();
}

// Bytes of the caller's input and output fields of a request.
size_t io_bytes(const cwo_params* p) { return 16 * (size_t)p->nx * p->ny; }

// Bytes a request holds from admission to completion when it runs alone: its input and
// output fields and its padded scratch plane.
size_t footprint(const cwo_params* p) {
    const Geometry g = geometry(p);
    return io_bytes(p) + elem_bytes(p->precision) * (size_t)g.ny * g.mx;
}

// Device memory the context holds: twiddle tables and every workspace.
size_t held_bytes(cwo_ctx* c) {
    size_t h = c->twiddle_bytes.load() + c->ws.held();
    for (const Slot& sl : c->slots) h += sl.ws.held();
    return h;
}

// Requests of one serving batch that do not touch each other's buffers are independent;
// such a batch is reordered (stably) so that requests of one geometry sit next to each
// other, those on one field first among them: run_jobs then runs them as shared-launch
// batches or z-stacks. A batch with a dependence keeps its arrival order.
// Requests that can share a serving batch's launches: one geometry and storage.
bool same_geometry(const cwo_job& a, const cwo_job& b) {
    return a.p.nx == b.p.nx && a.p.ny == b.p.ny && a.p.dx == b.p.dx && a.p.dy == b.p.dy &&
           a.p.flags == b.p.flags && a.p.precision == b.p.precision;
}

void group_batch(std::vector<cwo_job>& batch, std::vector<uint64_t>& ids) {
    const size_t n = batch.size();
    for (size_t i = 0; i < n; ++i)
        for (size_t j = 0; j < n; ++j)
            if (i != j && (batch[i].out == batch[j].in || batch[i].out == batch[j].out)) return;
    std::vector<size_t> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = i;
    auto key = [&](size_t i) {
        const cwo_params& p = batch[i].p;
        return std::make_tuple(p.nx, p.ny, p.dx, p.dy, p.flags, p.precision,
                               reinterpret_cast<uintptr_t>(batch[i].in));
    };
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return key(a) < key(b); });
    std::vector<cwo_job> jb(n);
    std::vector<uint64_t> ib(n);
    for (size_t i = 0; i < n; ++i) {
        jb[i] = batch[order[i]];
        ib[i] = ids[order[i]];
    }
    batch.swap(jb);
    ids.swap(ib);
}

void serve_loop(cwo_ctx* c) {
    (void)hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(c->qmu);
    while (true) {
        // 1. retire finished batches
        bool any_running = false;
        for (Slot& sl : c->slots) {
            if (sl.running.empty()) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) {
                any_running = true;
                continue;
            }
            const double t = now_s(c);
            for (uint64_t id : sl.running) {
                auto it = c->tickets.find(id);
                if (it == c->tickets.end()) continue;
                it->second.state = (q == hipSuccess) ? 2 : CWO_ERR_DEVICE;
                it->second.t_done = t;
                c->reserved -= io_bytes(&it->second.job.p);
                if (it->second.ready) {
                    c->ready_pool.push_back(it->second.ready);
                    it->second.ready = nullptr;
                }
            }
            if (q != hipSuccess) c->sticky = CWO_ERR_DEVICE;
            sl.running.clear();
        }
        // 2. admit and launch
        for (Slot& sl : c->slots) {
            if (!sl.running.empty() || c->queue.empty()) continue;
            std::vector<cwo_job> batch;
            std::vector<uint64_t> ids;
            std::vector<size_t> taken;  // queue positions of the batch, ascending
            size_t io = 0, planes = 0;
            bool trimmed = false;
            const cwo_job& head = c->tickets[c->queue.front()].job;
            const bool head_batchable = batchable(head);
            for (size_t k = 0; k < c->queue.size() && k < c->serve_window &&
                               (int)batch.size() < c->serve_max_batch;
                 ++k) {
                const uint64_t id = c->queue[k];
                const Ticket& tk = c->tickets[id];
                if (k > 0) {
                    // a shared-launch batch, or a z-stack on the head's field
                    if (!(head_batchable && same_geometry(head, tk.job) && batchable(tk.job)) &&
                        !same_group(head, tk.job))
                        continue;
                    // not ahead of an earlier request left in the queue that shares a buffer
                    bool clash = false;
                    for (size_t e = 0, t = 0; e < k && !clash; ++e) {
                        if (t < taken.size() && taken[t] == e) {
                            ++t;
                            continue;
                        }
                        const cwo_job& o = c->tickets[c->queue[e]].job;
                        clash = o.out == tk.job.in || o.out == tk.job.out || o.in == tk.job.out;
                    }
                    if (clash) continue;
                    const size_t pb = footprint(&tk.job.p) - io_bytes(&tk.job.p);
                    if (planes + pb > c->serve_batch_bytes) break;
                }
                batch.push_back(tk.job);
                // the memory of the batch as it will run (grouped by geometry)
                std::vector<cwo_job> grouped = batch;
                std::vector<uint64_t> gids(batch.size(), 0);
                group_batch(grouped, gids);
                const WsNeed need = jobs_need(c, grouped.data(), (int)grouped.size());
                auto fits = [&] {
                    return !c->budget || c->reserved + io + io_bytes(&tk.job.p) + held_bytes(c) +
                                                 growth(sl.ws, need) <=
                                             c->budget;
                };
                bool ok = fits();
                if (!ok && !trimmed) {
                    // give back the workspaces of idle slots (this one included) and retry
                    trimmed = true;
                    for (Slot& o : c->slots)
                        if (o.running.empty() && o.ws.held() > 0) o.ws.release();
                    ok = fits();
                }
                if (!ok) {
                    batch.pop_back();
                    break;  // FIFO: the next request waits for memory
                }
                io += io_bytes(&tk.job.p);
                planes += footprint(&tk.job.p) - io_bytes(&tk.job.p);
                ids.push_back(id);
                taken.push_back(k);
            }
            if (batch.empty()) {
                // the head does not fit; with nothing running and nothing left to give back it
                // never will (the synchronous calls' workspace holds the rest)
                bool busy = false;
                for (const Slot& o : c->slots) busy = busy || !o.running.empty();
                if (!busy) {
                    const uint64_t id = c->queue.front();
                    c->queue.pop_front();
                    Ticket& tk = c->tickets[id];
                    tk.state = CWO_ERR_NOMEM;
                    tk.t_done = now_s(c);
                    if (tk.ready) {
                        c->ready_pool.push_back(tk.ready);
                        tk.ready = nullptr;
                    }
                    continue;
                }
                break;
            }
            for (size_t t = taken.size(); t-- > 0;) c->queue.erase(c->queue.begin() + taken[t]);
            group_batch(batch, ids);
            const double t = now_s(c);
            std::vector<hipEvent_t> waits;
            for (uint64_t id : ids) {
                Ticket& tk = c->tickets[id];
                tk.state = 1;
                tk.t_start = t;
                if (tk.ready) waits.push_back(tk.ready);
            }
            c->reserved += io;
            sl.running = ids;  // the slot is busy from here on (drain waits for it)
            any_running = true;
            // launch without the queue lock: allocations and launches do not block submit/poll
            lk.unlock();
            cwo_status st;
            {
                std::lock_guard<std::mutex> g(c->mu);  // twiddle tables, profiling state
                st = c->sticky;
                for (hipEvent_t e : waits)
                    if (st == CWO_OK && hipStreamWaitEvent(sl.stream, e, 0) != hipSuccess)
                        st = dev_fail(c);
                if (st == CWO_OK) st = run_jobs(c, sl.ws, batch.data(), (int)batch.size(), sl.stream);
                if (st == CWO_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess) st = dev_fail(c);
            }
            lk.lock();
            if (st != CWO_OK) {
                // nothing of the batch may still run when its tickets report an error
                (void)hipStreamSynchronize(sl.stream);
                for (uint64_t id : ids) {
                    Ticket& tk = c->tickets[id];
                    tk.state = st;
                    tk.t_done = now_s(c);
                    c->reserved -= io_bytes(&tk.job.p);
                    if (tk.ready) {
                        c->ready_pool.push_back(tk.ready);
                        tk.ready = nullptr;
                    }
                }
                sl.running.clear();
            }
        }
        c->qcv.notify_all();  // progress for drain()
        if (c->stop && c->queue.empty() && !any_running) break;
        if (any_running)
            c->qcv.wait_for(lk, std::chrono::microseconds(c->serve_poll_us));
        else
            c->qcv.wait(lk, [&] { return c->stop || !c->queue.empty(); });
    }
}

cwo_status start_serving(cwo_ctx* c) {
    if (c->worker.joinable()) return CWO_OK;
    if (hipSetDevice(c->device) != hipSuccess) return dev_fail(c);
    for (Slot& sl : c->slots) {
        // default priority streams
        if (!sl.stream && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
            return dev_fail(c);
        if (!sl.done && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
            return dev_fail(c);
        sl.ws.owner = sl.stream;
    }
    c->slots_ready = true;
    c->stop = false;
    c->worker = std::thread(serve_loop, c);
    return CWO_OK;
}

void stop_serving(cwo_ctx* c) {
    {
        std::lock_guard<std::mutex> lk(c->qmu);
        c->stop = true;
    }
    c->qcv.notify_all();
    if (c->worker.joinable()) c->worker.join();
}

// Fresnel Fourier form: sizes as the other kinds, z != 0, no flags, complex64 only.
cwo_status validate_fourier(const cwo_params* p) {
    if (!p) return CWO_ERR_INVALID;
    if (p->kind != 0 && p->kind != CWO_FRESNEL_FOURIER) return CWO_ERR_INVALID;
    if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->wavelength)) return CWO_ERR_INVALID;
    if (!std::isfinite(p->z) || p->z == 0.0) return CWO_ERR_INVALID;
    if (p->flags != 0) return CWO_ERR_INVALID;
    if (p->precision < CWO_PREC_F32 || p->precision > CWO_PREC_BF16_STORAGE) return CWO_ERR_INVALID;
    if (!is_pow2(p->nx) || !is_pow2(p->ny) || p->nx < kMinN || p->ny < kMinN || p->nx > kMaxN ||
        p->ny > kMaxN)
        return CWO_ERR_UNSUPPORTED;
    if (p->precision != CWO_PREC_F32) return CWO_ERR_UNSUPPORTED;
    return CWO_OK;
}

// Shifted Fresnel: sizes as the other kinds (padded 2N), z != 0, no flags, complex64 only.
cwo_status validate_sfresnel(const cwo_params* p, const cwo_sfresnel* w) {
    if (!p || !w) return CWO_ERR_INVALID;
    if (p->kind != 0 && p->kind != CWO_FRESNEL_SHIFTED) return CWO_ERR_INVALID;
    if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->wavelength)) return CWO_ERR_INVALID;
    if (!finite_pos(w->dx1) || !finite_pos(w->dy1)) return CWO_ERR_INVALID;
    for (double v : {w->ox0, w->oy0, w->ox1, w->oy1})
        if (!std::isfinite(v)) return CWO_ERR_INVALID;
    if (!std::isfinite(p->z) || p->z == 0.0) return CWO_ERR_INVALID;
    if (p->flags != 0) return CWO_ERR_INVALID;
    if (p->precision < CWO_PREC_F32 || p->precision > CWO_PREC_BF16_STORAGE) return CWO_ERR_INVALID;
    if (!is_pow2(p->nx) || !is_pow2(p->ny) || p->nx < kMinN || p->ny < kMinN || p->nx > kMaxN ||
        p->ny > kMaxN)
        return CWO_ERR_UNSUPPORTED;
    if (p->precision != CWO_PREC_F32) return CWO_ERR_UNSUPPORTED;
    return CWO_OK;
}

// Epilogues: stream-ordered elementwise passes on the context's device.
template <class F>
cwo_status epilogue(cwo_ctx* c, size_t n, bool ok, F&& launch) {
    if (!c || !ok) return CWO_ERR_INVALID;
    if (n == 0) return CWO_OK;
    std::lock_guard<std::mutex> lock(c->mu);
    const cwo_status st = begin(c);
    if (st != CWO_OK) return st;
    CWO_HIP(c, launch());
    return CWO_OK;
}

// ---- scratch of the no-allocation entry point ------------------------------------------
// cwo_asm_noalloc keeps its twiddle tables and its padded plane in one statically
// allocated device array instead of memory it would have to allocate: up to 2 * 8192
// twiddles, then a plane of at most 64 MiB (ny * 2nx complex64, i.e. fields up to
// 2048 x 2048). Every device the library runs on holds its own copy until the process ends.
constexpr size_t kStaticTwiddleBytes = 2 * sizeof(float2) * 8192;
constexpr size_t kStaticPlaneBytes = size_t(64) << 20;
constexpr size_t kStaticScratchBytes = kStaticTwiddleBytes + kStaticPlaneBytes;
constexpr int kMaxDevices = 64;

// On the host this name stands for the array, not for its device address: kernels and
// copies take the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_static_mu;
void* g_static_addr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device; looked up
// once per device (cwo_create does it), then reused.
void* static_scratch(int device, cwo_status* st) {
    if (device < 0 || device >= kMaxDevices) {
        *st = CWO_ERR_UNSUPPORTED;
        return nullptr;
    }
    std::lock_guard<std::mutex> g(g_static_mu);
    if (!g_static_addr[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            *st = CWO_ERR_DEVICE;
            return nullptr;
        }
        g_static_addr[device] = ptr;
    }
    return g_static_addr[device];
}

// after != nullptr: the job's first kernel waits for the work enqueued on that stream
// before the call (an event recorded there now); the event returns to the pool when the
// ticket finishes.
cwo_status submit_impl(cwo_ctx* c, const cwo_job* job, bool ordered, hipStream_t after,
                       uint64_t* ticket) {
    if (!c || !job || !ticket) return CWO_ERR_INVALID;
    const int kind = job->p.kind;
    cwo_status st = validate(&job->p, kind, true);
    if (st != CWO_OK) return st;
    if (!job->in || !job->out) return CWO_ERR_INVALID;
    const size_t fp = footprint(&job->p);
    if (c->budget && fp > c->budget) return CWO_ERR_NOMEM;
    std::lock_guard<std::mutex> lk(c->qmu);
    if (c->sticky != CWO_OK) return c->sticky;
    if (!c->worker.joinable() && (st = start_serving(c)) != CWO_OK) return st;
    hipEvent_t ready = nullptr;
    if (ordered) {
        if (!c->ready_pool.empty()) {
            ready = c->ready_pool.back();
            c->ready_pool.pop_back();
        } else if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) {
            return dev_fail(c);
        }
        if (hipEventRecord(ready, after) != hipSuccess) {
            c->ready_pool.push_back(ready);
            return dev_fail(c);
        }
    }
    const uint64_t id = c->next_ticket++;
    Ticket tk;
    tk.job = *job;
    tk.footprint = fp;
    tk.ready = ready;
    tk.t_submit = now_s(c);
    c->tickets.emplace(id, tk);
    c->queue.push_back(id);
    *ticket = id;
    c->qcv.notify_all();
    return CWO_OK;
}

}  // namespace

extern "C" {

cwo_status cwo_submit(cwo_ctx* c, const cwo_job* job, uint64_t* ticket) {
    return submit_impl(c, job, false, nullptr, ticket);
}

cwo_status cwo_submit_after(cwo_ctx* c, const cwo_job* job, void* hip_stream, uint64_t* ticket) {
    return submit_impl(c, job, true, (hipStream_t)hip_stream, ticket);
}

cwo_status cwo_memory_held(cwo_ctx* c, size_t* bytes) {
    if (!c || !bytes) return CWO_ERR_INVALID;
    *bytes = held_bytes(c);
    return CWO_OK;
}

cwo_status cwo_poll(cwo_ctx* c, uint64_t ticket, int32_t* state) {
    if (!c || !state) return CWO_ERR_INVALID;
    std::lock_guard<std::mutex> lk(c->qmu);
    auto it = c->tickets.find(ticket);
    if (it == c->tickets.end()) return CWO_ERR_NOTFOUND;
    *state = it->second.state;
    return CWO_OK;
}

cwo_status cwo_ticket_info(cwo_ctx* c, uint64_t ticket, cwo_ticket* info) {
    if (!c || !info) return CWO_ERR_INVALID;
    std::lock_guard<std::mutex> lk(c->qmu);
    auto it = c->tickets.find(ticket);
    if (it == c->tickets.end()) return CWO_ERR_NOTFOUND;
    info->state = it->second.state;
    info->t_submit = it->second.t_submit;
    info->t_start = it->second.t_start;
    info->t_done = it->second.t_done;
    info->footprint = it->second.footprint;
    return CWO_OK;
}

cwo_status cwo_release(cwo_ctx* c, uint64_t ticket) {
    if (!c) return CWO_ERR_INVALID;
    std::lock_guard<std::mutex> lk(c->qmu);
    auto it = c->tickets.find(ticket);
    if (it == c->tickets.end()) return CWO_ERR_NOTFOUND;
    if (it->second.state == 0 || it->second.state == 1) return CWO_ERR_INVALID;  // not finished
    c->tickets.erase(it);
    return CWO_OK;
}

cwo_status cwo_drain(cwo_ctx* c) {
    if (!c) return CWO_ERR_INVALID;
    std::unique_lock<std::mutex> lk(c->qmu);
    c->qcv.wait(lk, [&] {
        if (!c->queue.empty()) return false;
        for (const Slot& sl : c->slots)
            if (!sl.running.empty()) return false;
        return true;
    });
    return c->sticky;
}


cwo_status cwo_create(cwo_ctx** ctx, int device, size_t hbm_budget_bytes) {
    if (!ctx) return CWO_ERR_INVALID;
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return CWO_ERR_DEVICE;
    if (device < 0 || device >= n) return CWO_ERR_INVALID;
    if (hipSetDevice(device) != hipSuccess) return CWO_ERR_DEVICE;
    cwo_status st = CWO_OK;
    if (device < kMaxDevices && !static_scratch(device, &st)) return st;
    cwo_ctx* c = new cwo_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    c->ws.budget = hbm_budget_bytes;
    load_tune_cache(c);
    read_serve_env(c);
    *ctx = c;
    return CWO_OK;
}

cwo_status cwo_destroy(cwo_ctx* c) {
    if (!c) return CWO_ERR_INVALID;
    stop_serving(c);  // finishes every submitted request first
    {
        std::lock_guard<std::mutex> lock(c->mu);
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        (void)drain_profile(c);
        for (auto& kv : c->twiddles) (void)hipFree(kv.second);
        c->ws.release();
        for (Slot& sl : c->slots) {
            sl.ws.release();
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        for (hipEvent_t e : c->spare) (void)hipEventDestroy(e);
        for (hipEvent_t e : c->ready_pool) (void)hipEventDestroy(e);
        for (auto& kv : c->tickets)
            if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    }
    delete c;
    return CWO_OK;
}

cwo_status cwo_asm(cwo_ctx* c, const cwo_params* p, const void* in, void* out, void* stream) {
    return propagate(c, p, CWO_ANGULAR, in, out, stream);
}

cwo_status cwo_asm_noalloc(cwo_ctx* c, const cwo_params* p, const void* in, void* out,
                           void* stream) {
    if (!c) return CWO_ERR_INVALID;
    cwo_status st = validate(p, CWO_ANGULAR, false);  // complex64 storage only
    if (st != CWO_OK) return st;
    if (!in || !out) return CWO_ERR_INVALID;
    const Geometry g = geometry(p);
    if (sizeof(float2) * (size_t)g.ny * g.mx > kStaticPlaneBytes) return CWO_ERR_NOMEM;
    std::lock_guard<std::mutex> lock(c->mu);
    st = begin(c);
    if (st != CWO_OK) return st;
    unsigned char* base = (unsigned char*)static_scratch(c->device, &st);
    if (!base) return st;
    hipStream_t s = (hipStream_t)stream;
    // twiddles are regenerated on the caller's stream each call (the array keeps whatever
    // the last call on this device left there)
    float2* twx = (float2*)base;
    float2* twy = twx + g.mx;
    void* buf = base + kStaticTwiddleBytes;
    CWO_HIP(c, cwo::launch_twiddles(twx, g.mx, s));
    CWO_HIP(c, cwo::launch_twiddles(twy, g.my, s));
    cwo::Storage sto;
    sto.out_scale = 1.0f / ((float)g.mx * (float)g.my);
    sto.layout = cwo::tiled_ok(g.nx, g.ny, g.mx, g.my) ? 1 : 0;
    const cwo::AsmScalars a = asm_scalars(p, g, p->z);
    CWO_HIP(c, cwo::launch_row_fwd((const float2*)in, buf, g.nx, g.ny, g.mx, 1, 0, 0, sto, twx, s));
    CWO_HIP(c, cwo::launch_col_asm(buf, g.ny, g.my, g.mx, 1, 0, a, sto, twy, s));
    CWO_HIP(c, cwo::launch_row_inv(buf, (float2*)out, g.nx, g.ny, g.mx, 1, 0, 0, sto, twx, s));
    return CWO_OK;
}

cwo_status cwo_fresnel(cwo_ctx* c, const cwo_params* p, const void* in, void* out, void* stream) {
    return propagate(c, p, CWO_FRESNEL_CONV, in, out, stream);
}

cwo_status cwo_asm_intensity(cwo_ctx* c, const cwo_params* p, const void* in, float* out,
                             void* stream) {
    return propagate(c, p, CWO_ANGULAR, in, out, stream, nullptr, true);
}

cwo_status cwo_fresnel_intensity(cwo_ctx* c, const cwo_params* p, const void* in, float* out,
                                 void* stream) {
    return propagate(c, p, CWO_FRESNEL_CONV, in, out, stream, nullptr, true);
}

cwo_status cwo_fresnel_fourier(cwo_ctx* c, const cwo_params* p, const void* in, void* out,
                               void* stream) {
    if (!c) return CWO_ERR_INVALID;
    cwo_status st = validate_fourier(p);
    if (st != CWO_OK) return st;
    if (!in || !out) return CWO_ERR_INVALID;
    std::lock_guard<std::mutex> lock(c->mu);
    st = begin(c);
    if (st != CWO_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const float2* twx = twiddle_table(c, p->nx, s, &st);
    if (!twx) return st;
    const float2* twy = twiddle_table(c, p->ny, s, &st);
    if (!twy) return st;
    float2* tabs = (float2*)ensure(c, c->ws, c->ws.fourier,
                                   sizeof(float2) * 2 * (size_t)(p->nx + p->ny), &st);
    if (!tabs) return st;
    cwo::FourierPlan fp;
    fp.nx = p->nx;
    fp.ny = p->ny;
    fp.dx = p->dx;
    fp.dy = p->dy;
    fp.dx2 = p->wavelength * p->z / ((double)p->nx * p->dx);
    fp.dy2 = p->wavelength * p->z / ((double)p->ny * p->dy);
    fp.inv2lz = 0.5 / (p->wavelength * p->z);
    fresnel_constant(p->dx, p->dy, p->wavelength, p->z, &fp.cre, &fp.cim);
    CWO_HIP(c, timed(c, CWO_STAGE_ROW_FWD, s, [&] {
                return cwo::launch_fresnel_fourier((const float2*)in, (float2*)out, tabs, fp, twx,
                                                   twy, s);
            }));
    return CWO_OK;
}

cwo_status cwo_fresnel_fourier_pitch(const cwo_params* p, double* dx2, double* dy2) {
    const cwo_status st = validate_fourier(p);
    if (st != CWO_OK) return st;
    if (!dx2 || !dy2) return CWO_ERR_INVALID;
    *dx2 = p->wavelength * p->z / ((double)p->nx * p->dx);
    *dy2 = p->wavelength * p->z / ((double)p->ny * p->dy);
    return CWO_OK;
}

cwo_status cwo_fresnel_shifted(cwo_ctx* c, const cwo_params* p, const cwo_sfresnel* w,
                               const void* in, void* out, void* stream) {
    if (!c) return CWO_ERR_INVALID;
    cwo_status st = validate_sfresnel(p, w);
    if (st != CWO_OK) return st;
    if (!in || !out) return CWO_ERR_INVALID;
    std::lock_guard<std::mutex> lock(c->mu);
    st = begin(c);
    if (st != CWO_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Workspace& ws = c->ws;
    const Geometry g{p->nx, p->ny, 2 * p->nx, 2 * p->ny};
    const float2* twx = twiddle_table(c, g.mx, s, &st);
    if (!twx) return st;
    const float2* twy = twiddle_table(c, g.my, s, &st);
    if (!twy) return st;
    float2* buf = (float2*)ensure(c, ws, ws.scratch, sizeof(float2) * (size_t)g.ny * g.mx, &st);
    if (!buf) return st;
    float2* tabs = (float2*)ensure(c, ws, ws.fourier, sizeof(float2) * 2 * (size_t)(g.nx + g.ny),
                                   &st);
    if (!tabs) return st;
    // the convolution kernel exp(i pi S d^2), S = p0 p1/(lambda z), is the Fresnel impulse
    // response of pitch sqrt(p0 p1); its factors carry no constant
    const FresnelKey key{g.mx, g.nx, g.my, g.ny, std::sqrt(p->dx * w->dx1),
                         std::sqrt(p->dy * w->dy1), p->wavelength, p->z, true, false};
    const float2* hfac = factor_table(c, ws, key, s, &st);
    if (!hfac) return st;
    cwo::SfPlan sp;
    sp.nx = g.nx;
    sp.ny = g.ny;
    sp.px0 = p->dx;
    sp.py0 = p->dy;
    sp.px1 = w->dx1;
    sp.py1 = w->dy1;
    sp.ox0 = w->ox0;
    sp.oy0 = w->oy0;
    sp.ox1 = w->ox1;
    sp.oy1 = w->oy1;
    sp.inv_lz = 1.0 / (p->wavelength * p->z);
    fresnel_constant(p->dx, p->dy, p->wavelength, p->z, &sp.cre, &sp.cim);
    CWO_HIP(c, timed(c, CWO_STAGE_TABLES, s, [&] { return cwo::launch_sf_tables(tabs, sp, s); }));
    CWO_HIP(c, timed(c, CWO_STAGE_ROW_FWD, s, [&] {
                return cwo::launch_sf_row_fwd((const float2*)in, buf, g.nx, g.ny, tabs, twx, s);
            }));
    CWO_HIP(c, timed(c, CWO_STAGE_COL, s, [&] {
                return cwo::launch_col_fresnel(buf, g.ny, g.my, g.mx, 1, 0, hfac, hfac + g.mx,
                                               cwo::Storage{}, twy, s);
            }));
    const float scale = 1.0f / ((float)g.mx * (float)g.my);
    CWO_HIP(c, timed(c, CWO_STAGE_ROW_INV, s, [&] {
                return cwo::launch_sf_row_inv(buf, (float2*)out, g.nx, g.ny, scale, tabs, twx, s);
            }));
    return CWO_OK;
}

}  // extern "C"

namespace {

// Point-light-source sums: sizes 1..kPlsMaxN per axis (any, not only powers of two),
// finite positive pitches and wavelength, finite offsets, oz != 0.
constexpr int kPlsMaxN = 16384;

cwo_status validate_pls(const cwo_pls_params* p, const float* points, int32_t npoints,
                        const void* out) {
    if (!p) return CWO_ERR_INVALID;
    if (p->nx < 1 || p->ny < 1 || p->nx > kPlsMaxN || p->ny > kPlsMaxN) return CWO_ERR_UNSUPPORTED;
    if (!out || npoints < 0 || (npoints > 0 && !points)) return CWO_ERR_INVALID;
    if (points && (reinterpret_cast<uintptr_t>(points) & 15) != 0) return CWO_ERR_INVALID;
    if (!finite_pos(p->px) || !finite_pos(p->py) || !finite_pos(p->wavelength))
        return CWO_ERR_INVALID;
    if (!std::isfinite(p->ox) || !std::isfinite(p->oy) || !std::isfinite(p->oz) || p->oz == 0.0)
        return CWO_ERR_INVALID;
    return CWO_OK;
}

cwo_status pls_run(cwo_ctx* c, const cwo_pls_params* p, const float* points, int32_t npoints,
                   void* out, bool field, hipStream_t s) {
    if (!c) return CWO_ERR_INVALID;
    cwo_status st = validate_pls(p, points, npoints, out);
    if (st != CWO_OK) return st;
    std::lock_guard<std::mutex> lock(c->mu);
    if ((st = begin(c)) != CWO_OK) return st;
    void* work = ensure(c, c->ws, c->ws.pls, cwo::pls_work_bytes(npoints), &st);
    if (!work) return st;
    cwo::PlsParams pp;
    pp.nx = p->nx;
    pp.ny = p->ny;
    pp.px = p->px;
    pp.py = p->py;
    pp.lam = p->wavelength;
    pp.ox = p->ox;
    pp.oy = p->oy;
    pp.oz = p->oz;
    // exp(i k oz)/(i lambda oz), k oz reduced in revolutions in FP64
    const double t = p->oz / p->wavelength;
    const double ang = 2.0 * M_PI * (t - std::nearbyint(t));
    const double inv = 1.0 / (p->wavelength * p->oz);
    pp.cre = std::sin(ang) * inv;  // (cos + i sin)/i = sin - i cos
    pp.cim = -std::cos(ang) * inv;
    CWO_HIP(c, timed(c, CWO_STAGE_PLS, s, [&] {
                return cwo::launch_pls(points, npoints, work, out, field, pp, s);
            }));
    return CWO_OK;
}

}  // namespace

extern "C" {

cwo_status cwo_pls_cgh(cwo_ctx* c, const cwo_pls_params* p, const float* points, int32_t npoints,
                       float* out, void* stream) {
    return pls_run(c, p, points, npoints, out, false, (hipStream_t)stream);
}

cwo_status cwo_pls_field(cwo_ctx* c, const cwo_pls_params* p, const float* points,
                         int32_t npoints, void* out, void* stream) {
    return pls_run(c, p, points, npoints, out, true, (hipStream_t)stream);
}

cwo_status cwo_intensity(cwo_ctx* c, const void* in, void* out, size_t n, void* stream) {
    return epilogue(c, n, n == 0 || (in && out), [&] {
        return cwo::launch_intensity((const float2*)in, (float*)out, n, (hipStream_t)stream);
    });
}

cwo_status cwo_phase(cwo_ctx* c, const void* in, void* out, size_t n, void* stream) {
    return epilogue(c, n, n == 0 || (in && out), [&] {
        return cwo::launch_phase((const float2*)in, (float*)out, n, (hipStream_t)stream);
    });
}

cwo_status cwo_polar(cwo_ctx* c, const void* phase, const void* amp, void* out, size_t n,
                     void* stream) {
    return epilogue(c, n, n == 0 || (phase && out), [&] {
        return cwo::launch_polar((const float*)phase, (const float*)amp, (float2*)out, n,
                                 (hipStream_t)stream);
    });
}

cwo_status cwo_scale(cwo_ctx* c, const void* in, void* out, int32_t out_u8, float top, size_t n,
                     void* stream) {
    const bool ok = (n == 0 || (in && out)) && (out_u8 == 0 || out_u8 == 1) &&
                    std::isfinite(top) && top > 0.0f && (out_u8 == 0 || top <= 255.0f);
    if (!c || !ok) return CWO_ERR_INVALID;
    if (n == 0) return CWO_OK;
    std::lock_guard<std::mutex> lock(c->mu);
    cwo_status st = begin(c);
    if (st != CWO_OK) return st;
    float* work = (float*)ensure(c, c->ws, c->ws.ework, sizeof(float) * (4 + 2 * cwo::kRangeBlocks),
                                 &st);
    if (!work) return st;
    CWO_HIP(c, cwo::launch_scale((const float*)in, n, top, out_u8 == 1, out, work,
                                 (hipStream_t)stream));
    return CWO_OK;
}

cwo_status cwo_asm_shifted(cwo_ctx* c, const cwo_params* p, const cwo_shift* sh, const void* in,
                           void* out, void* stream) {
    if (!c || !p || !sh) return CWO_ERR_INVALID;
    for (double v : {sh->ox, sh->oy, sh->cx, sh->wx, sh->cy, sh->wy})
        if (!std::isfinite(v)) return CWO_ERR_INVALID;
    cwo_status st = validate(p, CWO_ANGULAR, true);
    if (st != CWO_OK) return st;
    const cwo::AsmShift shift{sh->ox, sh->oy, sh->cx, sh->wx, sh->cy, sh->wy};
    return propagate(c, p, CWO_ANGULAR, in, out, stream, &shift);
}

cwo_status cwo_band_limit(const cwo_params* p, cwo_shift* sh) {
    if (!p || !sh) return CWO_ERR_INVALID;
    const cwo_status st = validate(p, CWO_ANGULAR, true);
    if (st != CWO_OK) return st;
    const Geometry g = geometry(p);
    auto width = [&](int m, double d) {
        const double df = 1.0 / ((double)m * d);
        const double t = 2.0 * df * p->z;
        return 2.0 / (p->wavelength * std::sqrt(t * t + 1.0));
    };
    *sh = cwo_shift{0.0, 0.0, 0.0, width(g.mx, p->dx), 0.0, width(g.my, p->dy)};
    return CWO_OK;
}

cwo_status cwo_autotune(cwo_ctx* c, const cwo_params* p, int32_t nz, const void* in, void* out,
                        void* stream, cwo_tuning* best) {
    if (!c || !p || !in || !out || nz < 1) return CWO_ERR_INVALID;
    const int kind = p->kind;
    cwo_status st = validate(p, kind, true);  // 16-bit storage: single planes and z-stacks
    if (st != CWO_OK) return st;
    std::lock_guard<std::mutex> lock(c->mu);
    st = begin(c);
    if (st != CWO_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const Geometry g = geometry(p);
    const bool half = !(p->flags & CWO_FLAG_NOPAD);
    std::vector<int> forms = (half && g.mx >= 1024) ? std::vector<int>{1, 2} : std::vector<int>{0};
    // single planes: the row-major and the tiled plane where tiles are possible (the tiled
    // row passes have one form)
    std::vector<int> layouts{0};
    if (nz == 1 && tiles_possible(g)) layouts = {1, 2};
    std::vector<int> chunks{0};
    if (nz > 1) {
        chunks.clear();
        for (int k : {2, 4, 8, 16, 32, cwo::kZChunk})
            if (k < nz || k == cwo::kZChunk) chunks.push_back(std::min(k, nz));
    }
    const TuneKey key = tune_key(p, kind, nz);
    std::vector<double> zs((size_t)nz, p->z);
    std::vector<void*> outs((size_t)nz);
    const size_t plane_bytes = sizeof(float2) * (size_t)p->nx * p->ny;
    for (int k = 0; k < nz; ++k) outs[k] = (char*)out + k * plane_bytes;
    auto run = [&]() {
        return nz == 1 ? propagate_locked(c, c->ws, p, kind, in, out, s)
                       : zstack_locked(c, c->ws, p, kind, zs.data(), nz, in, outs.data(), s);
    };
    hipEvent_t a = take_event(c), b = take_event(c);
    cwo_tuning found{0, 0, 0.0f, 0, 0};
    float best_ms = -1.0f;
    // (layout, row form, column form): the tiled plane has one row form and, for padded
    // columns of 4096 or 8192, two column forms
    struct Cand {
        int layout, row_form, col_form;
    };
    std::vector<Cand> cands;
    for (int lay : layouts) {
        if (lay == 2) {
            if (col_forms_possible(g, 1))
                for (int cf : {1, 2}) cands.push_back({lay, 0, cf});
            else
                cands.push_back({lay, 0, 0});
        } else {
            for (int f : forms) cands.push_back({lay, f, 0});
        }
    }
    for (const Cand& cd : cands) {
        const int f = cd.row_form;
        for (int zc : chunks) {
            const cwo_tuning cand{f, zc, 0.0f, cd.layout, cd.col_form};
            set_tuned(c, key, &cand);
            st = run();  // warm-up: allocations and tables
            if (st != CWO_OK) break;
            constexpr int kReps = 3;
            if (hipEventRecord(a, s) != hipSuccess) { st = dev_fail(c); break; }
            for (int r = 0; r < kReps && st == CWO_OK; ++r) st = run();
            if (st != CWO_OK) break;
            float ms = 0.0f;
            if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                hipEventElapsedTime(&ms, a, b) != hipSuccess) {
                st = dev_fail(c);
                break;
            }
            ms /= kReps;
            if (best_ms < 0.0f || ms < best_ms) {
                best_ms = ms;
                found = cwo_tuning{f, zc, (float)(1000.0 * ms / nz), cd.layout, cd.col_form};
            }
        }
        if (st != CWO_OK) break;
    }
    c->spare.push_back(a);
    c->spare.push_back(b);
    if (st != CWO_OK) {
        set_tuned(c, key, nullptr);
        return st;
    }
    set_tuned(c, key, &found);
    save_tune_cache(c);
    if (best) *best = found;
    return CWO_OK;
}

cwo_status cwo_set_tuning(cwo_ctx* c, const cwo_params* p, int32_t nz, const cwo_tuning* t) {
    if (!c || !p || nz < 1) return CWO_ERR_INVALID;
    const int kind = p->kind;
    cwo_status st = validate_geometry(p, kind, nz == 1);
    if (st != CWO_OK) return st;
    const TuneKey key = tune_key(p, kind, nz);
    if (!t) {
        set_tuned(c, key, nullptr);
        return CWO_OK;
    }
    if (t->row_form < 0 || t->row_form > 2 || t->zchunk < 0 || t->zchunk > cwo::kZChunk ||
        t->layout < 0 || t->layout > 2 || t->col_form < 0 || t->col_form > 2 ||
        !(t->us_per_plane >= 0.0f))
        return CWO_ERR_INVALID;
    const Geometry g = geometry(p);
    if (t->layout == 2 && !(nz == 1 && tiles_possible(g))) return CWO_ERR_UNSUPPORTED;
    if (t->col_form != 0 && !(nz == 1 && col_forms_possible(g, plane_layout(g, *t))))
        return CWO_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(c->mu);
    set_tuned(c, key, t);
    return CWO_OK;
}

cwo_status cwo_zstack(cwo_ctx* c, const cwo_params* p, const double* z, int32_t nz, const void* in,
                      void* out, void* stream) {
    if (!c || !p || !z || !in || !out || nz < 1) return CWO_ERR_INVALID;
    const int kind = p->kind;
    cwo_status st = validate_geometry(p, kind, true);  // 16-bit storage: padded planes
    if (st != CWO_OK) return st;
    for (int k = 0; k < nz; ++k)
        if ((st = validate_z(z[k], kind)) != CWO_OK) return st;
    const Geometry g = geometry(p);
    std::vector<void*> outs((size_t)nz);
    for (int k = 0; k < nz; ++k) outs[k] = (float2*)out + (size_t)k * g.ny * g.nx;
    std::lock_guard<std::mutex> lock(c->mu);
    if ((st = begin(c)) != CWO_OK) return st;
    return zstack_locked(c, c->ws, p, kind, z, nz, in, outs.data(), (hipStream_t)stream);
}

cwo_status cwo_batch(cwo_ctx* c, const cwo_job* jobs, int32_t njobs, void* stream) {
    if (!c || (!jobs && njobs > 0) || njobs < 0) return CWO_ERR_INVALID;
    cwo_status st = validate_jobs(jobs, njobs);
    if (st != CWO_OK) return st;
    std::lock_guard<std::mutex> lock(c->mu);
    if ((st = begin(c)) != CWO_OK) return st;
    return run_jobs(c, c->ws, jobs, njobs, (hipStream_t)stream);
}

cwo_status cwo_gs(cwo_ctx* c, const cwo_params* p, const float* a1, const float* a2, void* u,
                  int32_t iterations, float* errors, void* stream) {
    if (!c || !a1 || !a2 || !u || iterations < 0) return CWO_ERR_INVALID;
    cwo_status st = validate(p, CWO_ANGULAR, true);
    if (st != CWO_OK) return st;
    std::lock_guard<std::mutex> lock(c->mu);
    if ((st = begin(c)) != CWO_OK) return st;
    if (iterations == 0) return CWO_OK;
    hipStream_t s = (hipStream_t)stream;
    const Geometry g = geometry(p);
    const float2* twx = twiddle_table(c, g.mx, s, &st);
    if (!twx) return st;
    const float2* twy = twiddle_table(c, g.my, s, &st);
    if (!twy) return st;
    void* spec = ensure(c, c->ws, c->ws.scratch, elem_bytes(p->precision) * (size_t)g.ny * g.mx, &st);
    if (!spec) return st;
    double* num = nullptr;
    const size_t nrow = (size_t)g.ny * cwo::gs_partials(g.mx);  // error partials per iteration
    if (errors) {
        num = (double*)ensure(c, c->ws, c->ws.gsnum, sizeof(double) * ((size_t)iterations * nrow + cwo::kGsDenParts),
                              &st);
        if (!num) return st;
    }
    const cwo::AsmScalars fwd = asm_scalars(p, g, p->z), back = asm_scalars(p, g, -p->z);
    float2* field = (float2*)u;
    const size_t count = (size_t)g.ny * g.nx;
    // Storage of the padded spectrum; low precision takes the scalings of a single
    // propagation, and FP16 also scales each field entering a forward transform by 2^-e,
    // e the exponent of its largest component: the start field, then the amplitude that
    // constrained it (|a u/|u|| = a).
    cwo::Storage sto;
    cwo::GsScale g2, g1;  // row passes after the +z and the -z column pass
    sto.out_scale = 1.0f / ((float)g.mx * (float)g.my);
    g2.scale = g1.scale = sto.out_scale;
    // (the fused ping-pong row kernel has no split form: rows of 8192 stay row-major)
    sto.layout = g2.layout = g1.layout = cwo::tiled_ok(g.nx, g.ny, g.mx, g.my) && g.mx <= 4096 ? 1 : 0;
    if (p->precision != CWO_PREC_F32) {
        sto.prec = g2.prec = g1.prec = p->precision == CWO_PREC_F16_STORAGE ? 1 : 2;
        const int kx = ilog2(g.mx) / 2;
        sto.in_scale = g2.fwd_scale = g1.fwd_scale = std::ldexp(1.0f, -kx);
        sto.col_scale = 1.0f / (float)g.my;
        sto.out_scale = g2.scale = g1.scale = std::ldexp(1.0f, kx) / (float)g.mx;
        if (sto.prec == 1) {
            const size_t w = 2 + cwo::kRangeBlocks;
            float* rw = (float*)ensure(c, c->ws, c->ws.rwork, sizeof(float) * 3 * w, &st);
            if (!rw) return st;
            float *ru = rw, *ra2 = rw + w, *ra1 = rw + 2 * w;
            CWO_HIP(c, cwo::launch_range_scale(field, count, ru, s));
            CWO_HIP(c, cwo::launch_range_scale(a2, count, ra2, s));
            CWO_HIP(c, cwo::launch_range_scale(a1, count, ra1, s));
            sto.dyn_scale = ru;
            g2.dyn_fwd = ra2;
            g1.dyn_inv = ra2 + 1;
            g1.dyn_fwd = ra1;
            g2.dyn_inv = ru + 1;  // first iteration; ra1 + 1 from the second on
        }
    }
    CWO_HIP(c, timed(c, CWO_STAGE_ROW_FWD, s, [&] {
                return cwo::launch_row_fwd(field, spec, g.nx, g.ny, g.mx, 1, 0, 0, sto, twx, s);
            }));
    for (int k = 0; k < iterations; ++k) {
        CWO_HIP(c, timed(c, CWO_STAGE_COL, s, [&] {
                    return cwo::launch_col_asm(spec, g.ny, g.my, g.mx, 1, 0, fwd, sto, twy, s);
                }));
        double* nk = num ? num + (size_t)k * nrow : nullptr;
        CWO_HIP(c, timed(c, CWO_STAGE_ROW_GS, s, [&] {
                    return cwo::launch_row_gs(spec, a2, nullptr, nk, g.nx, g.ny, g.mx, g2, twx, s);
                }));
        CWO_HIP(c, timed(c, CWO_STAGE_COL, s, [&] {
                    return cwo::launch_col_asm(spec, g.ny, g.my, g.mx, 1, 0, back, sto, twy, s);
                }));
        float2* dst = (k == iterations - 1) ? field : nullptr;
        CWO_HIP(c, timed(c, CWO_STAGE_ROW_GS, s, [&] {
                    return cwo::launch_row_gs(spec, a1, dst, nullptr, g.nx, g.ny, g.mx, g1, twx, s);
                }));
        if (g1.dyn_fwd) g2.dyn_inv = g1.dyn_fwd + 1;
    }
    if (errors) {
        double* den = num + (size_t)iterations * nrow;
        CWO_HIP(c, cwo::launch_gs_errors(num, a2, den, errors, g.nx, g.ny, g.mx, iterations, s));
    }
    return CWO_OK;
}

cwo_status cwo_profile(cwo_ctx* c, int32_t enable) {
    if (!c) return CWO_ERR_INVALID;
    std::lock_guard<std::mutex> lock(c->mu);
    if (hipSetDevice(c->device) != hipSuccess || drain_profile(c) != hipSuccess) return dev_fail(c);
    if (enable) {
        for (int i = 0; i < CWO_STAGE_COUNT; ++i) {
            c->prof_ms[i] = 0.0;
            c->prof_n[i] = 0;
        }
    }
    c->profiling = enable != 0;
    return CWO_OK;
}

cwo_status cwo_profile_read(cwo_ctx* c, int32_t stage, double* total_ms, int64_t* launches) {
    if (!c || !total_ms || !launches || stage < 0 || stage >= CWO_STAGE_COUNT) return CWO_ERR_INVALID;
    std::lock_guard<std::mutex> lock(c->mu);
    if (hipSetDevice(c->device) != hipSuccess || drain_profile(c) != hipSuccess) return dev_fail(c);
    *total_ms = c->prof_ms[stage];
    *launches = c->prof_n[stage];
    return CWO_OK;
}

cwo_status cwo_check_params(const cwo_params* p, int32_t kind) {
    if (kind == CWO_FRESNEL_FOURIER) return validate_fourier(p);
    if (kind == CWO_FRESNEL_SHIFTED) {
        const cwo_sfresnel w{p ? p->dx : 1.0, p ? p->dy : 1.0, 0.0, 0.0, 0.0, 0.0};
        return validate_sfresnel(p, &w);
    }
    return validate(p, kind, true);
}

size_t cwo_scratch_bytes(const cwo_params* p) {
    if (!p) return 0;
    const int kind = p->kind == 0 ? CWO_ANGULAR : p->kind;
    if (validate(p, kind, true) != CWO_OK) return 0;
    const Geometry g = geometry(p);
    return elem_bytes(p->precision) * (size_t)g.ny * (size_t)g.mx;
}

const char* cwo_strerror(cwo_status s) {
    switch (s) {
        case CWO_OK: return "ok";
        case CWO_ERR_INVALID: return "invalid argument";
        case CWO_ERR_UNSUPPORTED: return "unsupported size or precision";
        case CWO_ERR_NOMEM: return "out of memory or over budget";
        case CWO_ERR_DEVICE: return "device error";
        case CWO_ERR_NOTFOUND: return "unknown ticket";
    }
    return "unknown status";
}

int32_t cwo_version(void) { return 100; }

}  // extern "C"
