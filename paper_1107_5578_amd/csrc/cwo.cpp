// Host runtime of libcwo: contexts, validation, tables, scratch and the C ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/cwo.h"
#include "launch.hpp"

namespace {

constexpr int kMinN = 16;
constexpr int kMaxN = 4096;
constexpr size_t kFresnelCacheEntries = 8;

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

struct FresnelKey {
    int mx, nx, my, ny;
    double dx, dy, lam, z;
    bool operator==(const FresnelKey& o) const {
        return mx == o.mx && nx == o.nx && my == o.my && ny == o.ny && dx == o.dx && dy == o.dy &&
               lam == o.lam && z == o.z;
    }
};

struct FresnelEntry {
    FresnelKey key;
    float2* h = nullptr;  // mx + my complex64: Hx (with C) then Hy
};

}  // namespace

struct cwo_ctx {
    int device = 0;
    size_t budget = 0;
    std::mutex mu;
    cwo_status sticky = CWO_OK;
    std::map<int, float2*> twiddles;  // FP32 exp(-2 pi i k / M) per M
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    double2* fres_work = nullptr;  // 2*M FP64 complex for the chirp transforms
    int fres_work_m = 0;
    std::list<FresnelEntry> fresnel;  // most recently used first
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
};

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

// Launch through `fn` (returning hipError_t); with profiling on, bracket it with events.
template <class F>
hipError_t timed(cwo_ctx* c, int stage, hipStream_t s, F&& fn) {
    if (!c->profiling) return fn();
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, s);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    c->recs.push_back({stage, a, b});
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

#define CWO_HIP(ctx, call)                          \
    do {                                            \
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
    return tw;
}

void* ensure_scratch(cwo_ctx* c, size_t bytes, cwo_status* st) {
    if (c->scratch_bytes >= bytes) return c->scratch;
    if (c->budget && bytes > c->budget) {
        *st = CWO_ERR_NOMEM;
        return nullptr;
    }
    if (c->scratch) {
        // the old buffer may still be read by queued kernels on any stream
        if (hipDeviceSynchronize() != hipSuccess) {
            *st = dev_fail(c);
            return nullptr;
        }
        (void)hipFree(c->scratch);
        c->scratch = nullptr;
        c->scratch_bytes = 0;
    }
    if (hipMalloc(&c->scratch, bytes) != hipSuccess) {
        c->scratch = nullptr;
        *st = CWO_ERR_NOMEM;
        return nullptr;
    }
    c->scratch_bytes = bytes;
    return c->scratch;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

cwo_status validate(const cwo_params* p, int kind) {
    if (!p) return CWO_ERR_INVALID;
    if (p->kind != 0 && p->kind != kind) return CWO_ERR_INVALID;
    if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->wavelength)) return CWO_ERR_INVALID;
    if (!std::isfinite(p->z)) return CWO_ERR_INVALID;
    if (kind == CWO_FRESNEL_CONV && p->z == 0.0) return CWO_ERR_INVALID;
    if ((p->flags & ~(uint32_t)CWO_FLAG_NOPAD) != 0) return CWO_ERR_INVALID;
    if (p->precision < CWO_PREC_F32 || p->precision > CWO_PREC_BF16_STORAGE) return CWO_ERR_INVALID;
    if (!is_pow2(p->nx) || !is_pow2(p->ny) || p->nx < kMinN || p->ny < kMinN || p->nx > kMaxN ||
        p->ny > kMaxN)
        return CWO_ERR_UNSUPPORTED;
    if (p->precision != CWO_PREC_F32) return CWO_ERR_UNSUPPORTED;
    return CWO_OK;
}

struct Geometry {
    int nx, ny, mx, my;
};

Geometry geometry(const cwo_params* p) {
    const bool nopad = (p->flags & CWO_FLAG_NOPAD) != 0;
    return Geometry{p->nx, p->ny, nopad ? p->nx : 2 * p->nx, nopad ? p->ny : 2 * p->ny};
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

const float2* fresnel_factors(cwo_ctx* c, const cwo_params* p, const Geometry& g, hipStream_t s,
                              cwo_status* st) {
    FresnelKey key{g.mx, g.nx, g.my, g.ny, p->dx, p->dy, p->wavelength, p->z};
    for (auto it = c->fresnel.begin(); it != c->fresnel.end(); ++it) {
        if (it->key == key) {
            c->fresnel.splice(c->fresnel.begin(), c->fresnel, it);
            return c->fresnel.front().h;
        }
    }
    const int mmax = g.mx > g.my ? g.mx : g.my;
    if (c->fres_work_m < mmax) {
        if (c->fres_work) {
            if (hipDeviceSynchronize() != hipSuccess) {
                *st = dev_fail(c);
                return nullptr;
            }
            (void)hipFree(c->fres_work);
            c->fres_work = nullptr;
            c->fres_work_m = 0;
        }
        if (hipMalloc(&c->fres_work, sizeof(double2) * 2 * (size_t)mmax) != hipSuccess) {
            *st = CWO_ERR_NOMEM;
            return nullptr;
        }
        c->fres_work_m = mmax;
    }
    FresnelEntry e;
    e.key = key;
    if (c->fresnel.size() >= kFresnelCacheEntries) {
        // reuse the least recently used buffer if it is large enough
        FresnelEntry old = c->fresnel.back();
        c->fresnel.pop_back();
        if (hipDeviceSynchronize() != hipSuccess) {
            *st = dev_fail(c);
            return nullptr;
        }
        (void)hipFree(old.h);
    }
    if (hipMalloc(&e.h, sizeof(float2) * (size_t)(g.mx + g.my)) != hipSuccess) {
        *st = CWO_ERR_NOMEM;
        return nullptr;
    }
    double cre, cim;
    fresnel_constant(p->dx, p->dy, p->wavelength, p->z, &cre, &cim);
    const double lz = p->wavelength * p->z;
    // the chirp work buffer is reused by consecutive launches on the same stream
    hipError_t herr = timed(c, CWO_STAGE_TABLES, s, [&] {
        hipError_t e1 = cwo::launch_fresnel_axis(c->fres_work, e.h, g.mx, g.nx, p->dx, lz, cre, cim, s);
        if (e1 != hipSuccess) return e1;
        return cwo::launch_fresnel_axis(c->fres_work, e.h + g.mx, g.my, g.ny, p->dy, lz, 1.0, 0.0, s);
    });
    if (herr != hipSuccess) {
        (void)hipFree(e.h);
        *st = dev_fail(c);
        return nullptr;
    }
    c->fresnel.push_front(e);
    return e.h;
}

cwo_status propagate(cwo_ctx* c, const cwo_params* p, int kind, const void* in, void* out,
                     void* stream) {
    if (!c) return CWO_ERR_INVALID;
    cwo_status st = validate(p, kind);
    if (st != CWO_OK) return st;
    if (!in || !out) return CWO_ERR_INVALID;
    std::lock_guard<std::mutex> lock(c->mu);
    if (c->sticky != CWO_OK) return c->sticky;
    CWO_HIP(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const Geometry g = geometry(p);
    const float2* twx = twiddle_table(c, g.mx, s, &st);
    if (!twx) return st;
    const float2* twy = twiddle_table(c, g.my, s, &st);
    if (!twy) return st;
    float2* buf = (float2*)ensure_scratch(c, sizeof(float2) * (size_t)g.ny * g.mx, &st);
    if (!buf) return st;
    const float2* fin = (const float2*)in;
    float2* fout = (float2*)out;
    CWO_HIP(c, timed(c, CWO_STAGE_ROW_FWD, s, [&] {
                return cwo::launch_row_fwd(fin, buf, g.nx, g.ny, g.mx, 1, 0, 0, twx, s);
            }));
    if (kind == CWO_ANGULAR) {
        cwo::AsmScalars a;
        a.dfx = 1.0 / ((double)g.mx * p->dx);
        a.dfy = 1.0 / ((double)g.my * p->dy);
        a.lam = p->wavelength;
        a.zl = p->z / p->wavelength;
        CWO_HIP(c, timed(c, CWO_STAGE_COL, s, [&] {
                    return cwo::launch_col_asm(buf, g.ny, g.my, g.mx, 1, 0, a, twy, s);
                }));
    } else {
        const float2* h = fresnel_factors(c, p, g, s, &st);
        if (!h) return st;
        CWO_HIP(c, timed(c, CWO_STAGE_COL, s, [&] {
                    return cwo::launch_col_fresnel(buf, g.ny, g.my, g.mx, 1, 0, h, h + g.mx, twy, s);
                }));
    }
    const float scale = 1.0f / ((float)g.mx * (float)g.my);  // power of two: exact
    CWO_HIP(c, timed(c, CWO_STAGE_ROW_INV, s, [&] {
                return cwo::launch_row_inv(buf, fout, g.nx, g.ny, g.mx, 1, 0, 0, scale, twx, s);
            }));
    return CWO_OK;
}

}  // namespace

extern "C" {

cwo_status cwo_create(cwo_ctx** ctx, int device, size_t hbm_budget_bytes) {
    if (!ctx) return CWO_ERR_INVALID;
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return CWO_ERR_DEVICE;
    if (device < 0 || device >= n) return CWO_ERR_INVALID;
    if (hipSetDevice(device) != hipSuccess) return CWO_ERR_DEVICE;
    cwo_ctx* c = new cwo_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    *ctx = c;
    return CWO_OK;
}

cwo_status cwo_destroy(cwo_ctx* c) {
    if (!c) return CWO_ERR_INVALID;
    {
        std::lock_guard<std::mutex> lock(c->mu);
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        for (auto& kv : c->twiddles) (void)hipFree(kv.second);
        for (auto& e : c->fresnel) (void)hipFree(e.h);
        if (c->scratch) (void)hipFree(c->scratch);
        if (c->fres_work) (void)hipFree(c->fres_work);
        (void)drain_profile(c);
        for (hipEvent_t e : c->spare) (void)hipEventDestroy(e);
    }
    delete c;
    return CWO_OK;
}

cwo_status cwo_asm(cwo_ctx* c, const cwo_params* p, const void* in, void* out, void* stream) {
    return propagate(c, p, CWO_ANGULAR, in, out, stream);
}

cwo_status cwo_fresnel(cwo_ctx* c, const cwo_params* p, const void* in, void* out, void* stream) {
    return propagate(c, p, CWO_FRESNEL_CONV, in, out, stream);
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
    if (kind != CWO_ANGULAR && kind != CWO_FRESNEL_CONV) return CWO_ERR_INVALID;
    return validate(p, kind);
}

size_t cwo_scratch_bytes(const cwo_params* p) {
    if (!p) return 0;
    const int kind = p->kind == 0 ? CWO_ANGULAR : p->kind;
    if (kind != CWO_ANGULAR && kind != CWO_FRESNEL_CONV) return 0;
    if (validate(p, kind) != CWO_OK) return 0;
    const Geometry g = geometry(p);
    return sizeof(float2) * (size_t)g.ny * (size_t)g.mx;
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
