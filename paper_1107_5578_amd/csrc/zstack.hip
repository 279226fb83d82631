// HIP kernels of the z-stack form (one field, many distances): the forward column
// transform once per column, then per plane the transfer function, the inverse column
// transform and the row inverse.

#include "kernel_common.hpp"

namespace cwo {

// ---- z-stack column pass ------------------------------------------------------
//
// One field, many distances: the forward column transform is done once per column
// and kept in registers; for each plane the spectrum is multiplied by that plane's
// transfer function and inverse transformed into the plane's scratch.

// The z-independent part of each bin is computed once, after the forward column
// transform, and kept across the plane loop; each plane then costs one FP64 multiply
// and a reduction per bin.
//
// Fast form (every bin s <= 0.05): K = 1 - sqrt(1 - s) = s/2 + T(s) from the same
// series as AsmHFast; the phase of plane z is zl - zl*K revolutions, i.e.
// reduce(zl) - reduce(zl*K). Exact form: Q = sqrt(1 - s) in FP64 (Q < 0 marks an
// evanescent bin, s > 1, decided with the reference's operations); the phase is zl*Q.
struct AsmZFast {
    double lam_dfx, lam_dfy;
    int mx, my;
    __device__ __forceinline__ double bin(int p, int q) const {
        const double x = (double)(p < mx / 2 ? p : p - mx) * lam_dfx;
        const double y = (double)(q < my / 2 ? q : q - my) * lam_dfy;
        const double s = x * x + y * y;
        double poly = 715.0 / 65536.0;
        poly = fma(poly, s, 429.0 / 32768.0);
        poly = fma(poly, s, 33.0 / 2048.0);
        poly = fma(poly, s, 21.0 / 1024.0);
        poly = fma(poly, s, 7.0 / 256.0);
        poly = fma(poly, s, 5.0 / 128.0);
        poly = fma(poly, s, 1.0 / 16.0);
        poly = fma(poly, s, 1.0 / 8.0);
        return fma(s * s, poly, 0.5 * s);
    }
    __device__ __forceinline__ float2 at(double k, double zl, float c0) const {
        const double u = zl * k;
        float r = c0 - (float)(u - rint(u));
        r -= rintf(r);
        return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
    }
};

struct AsmZExact {
    double dfx, dfy, lam;
    int mx, my;
    __device__ __forceinline__ double bin(int p, int q) const {
#pragma clang fp contract(off)
        const double pp = (double)(p < mx / 2 ? p : p - mx);
        const double qq = (double)(q < my / 2 ? q : q - my);
        const double ax = lam * (pp * dfx);
        const double ay = lam * (qq * dfy);
        const double s = ay * ay + ax * ax;
        return (s <= 1.0) ? sqrt(1.0 - s) : -1.0;
    }
    __device__ __forceinline__ float2 at(double qv, double zl, float) const {
        if (qv < 0.0) return make_float2(0.f, 0.f);
        const double t = zl * qv;
        const float r = (float)(t - rint(t));
        return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
    }
};

template <class ZH>
struct ZSetAsm {
    ZH h;
    double zl[kZChunk];
    int nz;
};

struct ZSetFresnel {
    const float2* h;  // plane k: Hx (with C) at h + k*stride, Hy at h + k*stride + mx
    size_t stride;
    int mx, nz;
};

template <int M, bool HALF, class ST>
__device__ __forceinline__ void zcol_load(const typename ST::E* __restrict__ src, int ny, int mx,
                                          int j, bool active, float2 (&v)[1][ZColCfg<M>::E]) {
    using C = ZColCfg<M>;
    constexpr int E = C::E, T = C::T;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int y = j + r * T;
        const bool ld = active && (HALF ? (r < E / 2) : (y < ny));
        v[0][r] = ld ? ST::dec(src[(size_t)y * mx]) : make_float2(0.f, 0.f);
    }
}

// The z-stack planes are written column-major (element (y, x) of a plane at x*ny + y):
// each column is contiguous, so a wavefront stores whole cache lines. Lines of these
// planes are never read before they are written; row-major stores of single columns
// would leave partially written lines in L2. hscale (a power of two; 1 for complex64)
// multiplies the stored values.
template <int M, bool HALF, class ST>
__device__ __forceinline__ void zcol_store(typename ST::E* __restrict__ dst, int ny, int j,
                                           bool active, const float2 (&w)[1][ZColCfg<M>::E],
                                           float hscale) {
    using C = ZColCfg<M>;
    constexpr int E = C::E, T = C::T;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int y = j + r * T;
        const bool st = active && (HALF ? (r < E / 2) : (y < ny));
        if (st) dst[y] = ST::enc(make_float2(w[0][r].x * hscale, w[0][r].y * hscale));
    }
}

// The per-bin factor K of the thread's column is parked in LDS (each thread reads back
// only what it wrote, so no barrier is involved): registers hold the forward spectrum
// and the twiddles, which would not fit beside K at two waves per SIMD.
template <int M, bool HALF, class ZH, class ST>
__global__ __launch_bounds__(ZColCfg<M>::THREADS) void k_col_z_asm(
    const typename ST::E* __restrict__ spec, typename ST::E* __restrict__ zbuf, int ny, int mx,
    size_t zplane, ZSetAsm<ZH> zs, float hscale, const float2* __restrict__ tw) {
    using C = ZColCfg<M>;
    constexpr int E = C::E, T = C::T;
    __shared__ float2 lds[C::PAIRS * C::LDS_PAIR];
    __shared__ double kbl[C::PAIRS * M];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int col0 = blk * C::PAIRS + sub;
    const bool active = col0 < mx;
    const int col = active ? col0 : 0;
    float2* my_lds = lds + sub * C::LDS_PAIR;
    double* my_kb = kbl + sub * M;
    TwCache<M, E> twc;
    twc.load(j, tw);
    float2 v[1][E];
    zcol_load<M, HALF, ST>(spec + col, ny, mx, j, active, v);
    fft<M, E, 1, FWD>(v, my_lds, j, twc);
#pragma unroll
    for (int r = 0; r < E; ++r) my_kb[j + r * T] = zs.h.bin(col, j + r * T);
    for (int k = 0; k < zs.nz; ++k) {
        const double zl = zs.zl[k];
        const float c0 = (float)(zl - rint(zl));
        float2 w[1][E];
#pragma unroll
        for (int r = 0; r < E; ++r) w[0][r] = cmul(v[0][r], zs.h.at(my_kb[j + r * T], zl, c0));
        fft<M, E, 1, INV>(w, my_lds, j, twc);
        zcol_store<M, HALF, ST>(zbuf + (size_t)k * zplane + (size_t)col * ny, ny, j, active, w,
                                hscale);
    }
}

template <int M, bool HALF, class ST>
__global__ __launch_bounds__(ZColCfg<M>::THREADS) void k_col_z_fresnel(
    const typename ST::E* __restrict__ spec, typename ST::E* __restrict__ zbuf, int ny, int mx,
    size_t zplane, ZSetFresnel zs, float hscale, const float2* __restrict__ tw) {
    using C = ZColCfg<M>;
    constexpr int E = C::E, T = C::T;
    __shared__ float2 lds[C::PAIRS * C::LDS_PAIR];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int col0 = blk * C::PAIRS + sub;
    const bool active = col0 < mx;
    const int col = active ? col0 : 0;
    float2* my_lds = lds + sub * C::LDS_PAIR;
    TwCache<M, E> twc;
    twc.load(j, tw);
    float2 v[1][E];
    zcol_load<M, HALF, ST>(spec + col, ny, mx, j, active, v);
    fft<M, E, 1, FWD>(v, my_lds, j, twc);
    for (int k = 0; k < zs.nz; ++k) {
        const float2* hk = zs.h + (size_t)k * zs.stride;
        const float2 hx = hk[col];
        float2 w[1][E];
#pragma unroll
        for (int r = 0; r < E; ++r) w[0][r] = cmul(v[0][r], cmul(hx, hk[zs.mx + j + r * T]));
        fft<M, E, 1, INV>(w, my_lds, j, twc);
        zcol_store<M, HALF, ST>(zbuf + (size_t)k * zplane + (size_t)col * ny, ny, j, active, w,
                                hscale);
    }
}

// Row inverse of z-stack planes stored column-major (element (y, x) at x*ny + y, as the
// z-stack column pass writes them). The data are laid out like the columns of the
// column pass, so the same configuration applies: each thread transforms P adjacent
// rows, reading P contiguous elements (16 bytes) per position; rows are stored to the
// row-major outputs with the crop and the 1/(Mx*My) scale. Tiles of rows are taken in
// XCD-contiguous ranges, so the blocks that share an input cache line share an L2.
template <int M, bool HALF, class OUT, class ST>
__global__ __launch_bounds__(ColCfg<M>::THREADS) __attribute__((amdgpu_waves_per_eu(ColCfg<M>::WAVES_PER_EU))) void k_row_inv_t(
    const typename ST::E* __restrict__ in, OUT outs, int nx, int ny, int batch, size_t in_plane,
    float scale, const float* __restrict__ dyn_inv, const float2* __restrict__ tw) {
    using C = ColCfg<M>;
    constexpr int E = C::E, T = C::T, P = C::P;
    using SE = typename ST::E;
    using PK = Pack<SE, P>;
    if (dyn_inv) scale *= *dyn_inv;
    __shared__ float4 lds4[C::PAIRS * C::LDS_PAIR / 2];
    float2* lds = reinterpret_cast<float2*>(lds4);
    const int tid = threadIdx.x;
    const int pair = tid / T, j = tid % T;
    float2* my_lds = lds + pair * C::LDS_PAIR;
    TwCache<M, E> twc;
    twc.load(j, tw);
    const int ntiles = (ny + C::COLS - 1) / C::COLS;
    auto item = [&](int it) {
        // the thread's index, opaque to the compiler in each item of the persistent loop: the
        // addresses derived from it are recomputed per item instead of held (or spilled)
        int jt = j;
        asm volatile("" : "+v"(jt));
        const int pl = it / ntiles, tile = it - pl * ntiles;
        const int y0 = (tile * C::PAIRS + pair) * P;  // first row of this thread (ny is even)
        const bool active = y0 < ny;
        const SE* base = in + pl * in_plane + (active ? y0 : 0);
        float2 v[P][E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const PK t = *reinterpret_cast<const PK*>(base + (size_t)(jt + r * T) * ny);
#pragma unroll
            for (int p = 0; p < P; ++p) v[p][r] = ST::dec(t.e[p]);
        }
        fft<M, E, P, INV, C::SPLIT>(v, my_lds, jt, twc);
        int jo = j;
        asm volatile("" : "+v"(jo));
        if (active) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const size_t base = (size_t)(y0 + p) * nx;
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const int x = jo + r * T;
                    if (HALF ? (r < E / 2) : (x < nx))
                        outs.put(pl, base + x, make_float2(v[p][r].x * scale, v[p][r].y * scale));
                }
            }
        }
    };
    if constexpr (HALF) {
        const ItemRange ir = xcd_items(blockIdx.x, gridDim.x, ntiles * batch);
        for (int it = ir.first; it < ir.end; it += ir.step) item(it);
    } else {
        item(xcd_remap(blockIdx.x, gridDim.x));
    }
}

// ---- host launchers ------------------------------------------------------------

namespace {
template <class ST>
hipError_t row_inv_z_t(const void* zbuf, const ZChunk& zc, int nx, int ny, int mx, size_t zplane,
                       float scale, const float* dyn_inv, const float2* tw, hipStream_t s) {
    using SE = typename ST::E;
    OutTable t;
    for (int k = 0; k < kZChunk; ++k) t.out[k] = k < zc.nz ? zc.out[k] : nullptr;
    const bool half = (mx == 2 * nx);
    CWO_DISPATCH_M(mx, {
        using C = ColCfg<MM>;
        const int items = (ny + C::COLS - 1) / C::COLS * zc.nz;
        if (half) {
            auto k = k_row_inv_t<MM, true, OutTable, ST>;
            const int g = resident_blocks(k, C::THREADS, items);
            launch_kernel(k, dim3(g), dim3(C::THREADS), 0, s, (const SE*)zbuf, t, nx, ny,
                               zc.nz, zplane, scale, dyn_inv, tw);
        } else if constexpr (std::is_same_v<ST, StF32>) {
            launch_kernel((k_row_inv_t<MM, false, OutTable, ST>), dim3(items),
                               dim3(C::THREADS), 0, s, (const SE*)zbuf, t, nx, ny, zc.nz, zplane,
                               scale, dyn_inv, tw);
        } else {
            return hipErrorInvalidValue;
        }
    });
    return hipGetLastError();
}

template <class ZH, class ST>
hipError_t col_z_asm_t(const void* spec, void* zbuf, int ny, int my, int mx, size_t zplane,
                       const ZSetAsm<ZH>& zs, float hscale, const float2* tw, hipStream_t s) {
    using SE = typename ST::E;
    const bool half = (my == 2 * ny);
    CWO_DISPATCH_M(my, {
        using C = ZColCfg<MM>;
        dim3 grid((mx + C::COLS - 1) / C::COLS);
        if (half)
            launch_kernel((k_col_z_asm<MM, true, ZH, ST>), grid, dim3(C::THREADS), 0, s,
                               (const SE*)spec, (SE*)zbuf, ny, mx, zplane, zs, hscale, tw);
        else if constexpr (std::is_same_v<ST, StF32>)
            launch_kernel((k_col_z_asm<MM, false, ZH, ST>), grid, dim3(C::THREADS), 0, s,
                               (const SE*)spec, (SE*)zbuf, ny, mx, zplane, zs, hscale, tw);
        else
            return hipErrorInvalidValue;
    });
    return hipGetLastError();
}

template <class ST>
hipError_t col_z_fresnel_t(const void* spec, void* zbuf, int ny, int my, int mx, size_t zplane,
                           const ZSetFresnel& zs, float hscale, const float2* tw, hipStream_t s) {
    using SE = typename ST::E;
    const bool half = (my == 2 * ny);
    CWO_DISPATCH_M(my, {
        using C = ZColCfg<MM>;
        dim3 grid((mx + C::COLS - 1) / C::COLS);
        if (half)
            launch_kernel((k_col_z_fresnel<MM, true, ST>), grid, dim3(C::THREADS), 0, s,
                               (const SE*)spec, (SE*)zbuf, ny, mx, zplane, zs, hscale, tw);
        else if constexpr (std::is_same_v<ST, StF32>)
            launch_kernel((k_col_z_fresnel<MM, false, ST>), grid, dim3(C::THREADS), 0, s,
                               (const SE*)spec, (SE*)zbuf, ny, mx, zplane, zs, hscale, tw);
        else
            return hipErrorInvalidValue;
    });
    return hipGetLastError();
}

template <class ZH>
hipError_t col_z_asm_prec(const void* spec, void* zbuf, int ny, int my, int mx, size_t zplane,
                          const ZSetAsm<ZH>& zs, const Storage& st, const float2* tw,
                          hipStream_t s) {
    switch (st.prec) {
        case 0: return col_z_asm_t<ZH, StF32>(spec, zbuf, ny, my, mx, zplane, zs, st.col_scale, tw, s);
        case 1: return col_z_asm_t<ZH, StF16>(spec, zbuf, ny, my, mx, zplane, zs, st.col_scale, tw, s);
        case 2: return col_z_asm_t<ZH, StBF16>(spec, zbuf, ny, my, mx, zplane, zs, st.col_scale, tw, s);
    }
    return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_row_inv_z(const void* zbuf, const ZChunk& zc, int nx, int ny, int mx,
                            size_t zplane, const Storage& st, const float2* tw, hipStream_t s) {
    switch (st.prec) {
        case 0: return row_inv_z_t<StF32>(zbuf, zc, nx, ny, mx, zplane, st.out_scale, st.dyn_inv, tw, s);
        case 1: return row_inv_z_t<StF16>(zbuf, zc, nx, ny, mx, zplane, st.out_scale, st.dyn_inv, tw, s);
        case 2: return row_inv_z_t<StBF16>(zbuf, zc, nx, ny, mx, zplane, st.out_scale, st.dyn_inv, tw, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_col_z_asm(const void* spec, void* zbuf, int ny, int my, int mx, size_t zplane,
                            const AsmScalars& a, const ZChunk& zc, const Storage& st,
                            const float2* tw, hipStream_t s) {
    const double sx = a.lam * (0.5 * mx) * a.dfx, sy = a.lam * (0.5 * my) * a.dfy;
    if (sx * sx + sy * sy <= kAsmFastMaxS) {
        ZSetAsm<AsmZFast> zs;
        zs.h = AsmZFast{a.lam * a.dfx, a.lam * a.dfy, mx, my};
        for (int k = 0; k < kZChunk; ++k) zs.zl[k] = k < zc.nz ? zc.zl[k] : 0.0;
        zs.nz = zc.nz;
        return col_z_asm_prec(spec, zbuf, ny, my, mx, zplane, zs, st, tw, s);
    }
    ZSetAsm<AsmZExact> zs;
    zs.h = AsmZExact{a.dfx, a.dfy, a.lam, mx, my};
    for (int k = 0; k < kZChunk; ++k) zs.zl[k] = k < zc.nz ? zc.zl[k] : 0.0;
    zs.nz = zc.nz;
    return col_z_asm_prec(spec, zbuf, ny, my, mx, zplane, zs, st, tw, s);
}

hipError_t launch_col_z_fresnel(const void* spec, void* zbuf, int ny, int my, int mx,
                                size_t zplane, const float2* h, int nz, const Storage& st,
                                const float2* tw, hipStream_t s) {
    const ZSetFresnel zs{h, (size_t)(mx + my), mx, nz};
    switch (st.prec) {
        case 0: return col_z_fresnel_t<StF32>(spec, zbuf, ny, my, mx, zplane, zs, st.col_scale, tw, s);
        case 1: return col_z_fresnel_t<StF16>(spec, zbuf, ny, my, mx, zplane, zs, st.col_scale, tw, s);
        case 2: return col_z_fresnel_t<StBF16>(spec, zbuf, ny, my, mx, zplane, zs, st.col_scale, tw, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace cwo
