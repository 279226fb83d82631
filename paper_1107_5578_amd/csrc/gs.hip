// HIP kernels of the amplitude-constrained ping-pong iteration (the column pass is the
// plain one).

#include "kernel_common.hpp"

namespace cwo {

// ---- ping-pong iteration row kernel ----------------------------------------------
//
// Row inverse transform, crop, amplitude constraint and re-padded forward transform
// fused, so one propagation of the iteration is a column pass plus this kernel.
// ST is the storage of the padded spectrum. The stored rows carry a power-of-two factor:
// the inverse transform is multiplied by scale * (*dyn_inv) to give the physical field,
// and the constrained field by fwd_scale * (*dyn_fwd) before the forward transform (null
// dyn pointers count as 1), so FP16 storage stays in range.

// Error partials of one row: each thread's double summed over its wavefront's share of the
// row (the row's T threads are T consecutive lanes, or whole wavefronts when T >= 64) by a
// butterfly of cross-lane exchanges in a fixed order, and stored by the share's first lane
// at num[row * P + w], w the row's wavefront (P = max(1, T/64) partials per row). The
// iteration's error sums them later in a fixed order too, so it stays deterministic; no
// block barrier is taken here.
// All lanes of the wavefront call it (store: whether this row exists).
template <int T>
__device__ __forceinline__ void row_partials(double x, double* __restrict__ num, int row, int j,
                                             bool store) {
    constexpr int W = T < 64 ? T : 64;
    constexpr int P = T < 64 ? 1 : T / 64;
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (store && (j & (W - 1)) == 0) num[(size_t)row * P + j / W] = x;
}

// Error partials per row for rows of m points (the row kernels run m/16 threads per row).
constexpr int gs_partials_per_row(int m) { return m / 16 < 64 ? 1 : m / 16 / 64; }

template <int M, bool HALF, class ST>
__global__ __launch_bounds__(RowCfg<M>::THREADS) void k_row_gs(
    typename ST::E* __restrict__ spec, const float* __restrict__ amp, float2* __restrict__ out,
    double* __restrict__ num, int nx, int ny, float scale, const float* __restrict__ dyn_inv,
    float fwd_scale, const float* __restrict__ dyn_fwd, const float2* __restrict__ tw) {
    using C = RowCfg<M>;
    using SE = typename ST::E;
    constexpr int E = C::E, T = C::T;
    __shared__ float2 lds[C::RPB * lds_elems<M>()];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    const int row = blockIdx.x * C::RPB + sub;
    const bool valid = row < ny;
    SE* srow = spec + (size_t)(valid ? row : 0) * M;
    const float* arow = amp + (size_t)(valid ? row : 0) * nx;
    float2* my_lds = lds + sub * lds_elems<M>();
    if (dyn_inv) scale *= *dyn_inv;
    TwCache<M, E> twc;
    twc.load(j, tw);
    float2 v[1][E];
#pragma unroll
    for (int r = 0; r < E; ++r)
        v[0][r] = valid ? ST::dec(srow[j + r * T]) : make_float2(0.f, 0.f);
    fft<M, E, 1, INV>(v, my_lds, j, twc);
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = j + r * T;
        const bool in_field = HALF ? (r < E / 2) : (x < nx);
        if (in_field) {
            const float a = valid ? arow[x] : 0.f;
            const float re = v[0][r].x * scale, im = v[0][r].y * scale;
            const float m2 = re * re + im * im;
            float2 c;
            if (m2 > 0.f) {
                const float mag = __fsqrt_rn(m2);
                const float f = a / mag;
                c = make_float2(re * f, im * f);
                const double d = (double)mag - (double)a;
                acc += d * d;
            } else {
                c = make_float2(a, 0.f);
                acc += (double)a * (double)a;
            }
            v[0][r] = c;
        } else {
            v[0][r] = make_float2(0.f, 0.f);  // the padding of the next forward transform
        }
    }
    if (num) row_partials<T>(acc, num, row, j, valid);
    if (out) {
        if (valid) {
            float2* orow = out + (size_t)row * nx;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int x = j + r * T;
                if (HALF ? (r < E / 2) : (x < nx)) orow[x] = v[0][r];
            }
        }
        return;
    }
    if (dyn_fwd) fwd_scale *= *dyn_fwd;
    if (fwd_scale != 1.0f) {
#pragma unroll
        for (int r = 0; r < E; ++r) v[0][r] = make_float2(v[0][r].x * fwd_scale, v[0][r].y * fwd_scale);
    }
    if constexpr (HALF) fft_zpad<M, E, 1, FWD>(v, my_lds, j, twc);
    else fft<M, E, 1, FWD>(v, my_lds, j, twc);
    if (valid) {
#pragma unroll
        for (int r = 0; r < E; ++r) srow[j + r * T] = ST::enc(v[0][r]);
    }
}

// The same on the tiled spectrum plane (padded rows, Mx = 2Nx): groups of RPB rows per
// block, a resident grid (the blocks of one XCD take that XCD's contiguous range of
// groups), the next group's tile rows loaded into registers while the current group is
// processed. Per group: tile rows regrouped into rows in LDS, inverse transform, crop,
// constraint and the row's error partial; then either the constrained field to out, or
// the re-padded forward transform regrouped by tile and stored back in place (each block
// reads and writes only its own groups' tile rows).
// RPB rows per block
template <int M, int RPB_>
struct GsTileCfg {
    static constexpr int E = 16;
    static constexpr int T = M / E;
    static constexpr int RPB = RPB_;
    static constexpr int THREADS = T * RPB;
    static constexpr int TS = kTileW * RPB;
    static constexpr int XCH = RPB * lds_elems<M>();
    static constexpr int TRN = (M / kTileW) * TS;
    static constexpr int LDS = XCH > TRN ? XCH : TRN;
};
template <int M, int RPB, class SE>
struct GsTileChunks {
    using C = GsTileCfg<M, RPB>;
    static constexpr int CE = 16 / (int)sizeof(SE);
    static constexpr int PER_TILE = RPB * kTileW / CE;
    static constexpr int CPT = (M / kTileW) * PER_TILE / C::THREADS;
    static_assert(CPT * C::THREADS == (M / kTileW) * PER_TILE, "chunks");
};

template <int M, class ST, int RPB, int PF>
__global__ __launch_bounds__((GsTileCfg<M, RPB>::THREADS)) __attribute__((amdgpu_waves_per_eu(2))) void k_row_gs_tile(
    typename ST::E* __restrict__ spec, const float* __restrict__ amp, float2* __restrict__ out,
    double* __restrict__ num, int nx, int ny, float scale, const float* __restrict__ dyn_inv,
    float fwd_scale, const float* __restrict__ dyn_fwd, const float2* __restrict__ tw) {
    using C = GsTileCfg<M, RPB>;
    using SE = typename ST::E;
    using K = GsTileChunks<M, RPB, SE>;
    using PK = Pack<SE, K::CE>;
    constexpr int E = C::E, T = C::T, NL = E / 2;
    __shared__ float2 lds[C::LDS];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    float2* my_lds = lds + sub * lds_elems<M>();
    if (dyn_inv) scale *= *dyn_inv;
    if (dyn_fwd) fwd_scale *= *dyn_fwd;
    const int groups = ny / C::RPB;
    const ItemRange ir = xcd_items(blockIdx.x, gridDim.x, groups);
    TwCache<M, E> twc;
    twc.load(j, tw);
    auto load = [&](int g, PK (&d)[K::CPT], int tl, int lo, int hi) {
        const int y0 = g * C::RPB;
#pragma unroll
        for (int k = lo; k < hi; ++k) {
            const int c = tl + k * C::THREADS;
            const int t = c / K::PER_TILE, q = c - t * K::PER_TILE;
            d[k] = *reinterpret_cast<const PK*>(spec + ((size_t)t * ny + y0) * kTileW + q * K::CE);
        }
    };
    // the amplitudes of the thread's row are loaded with the group's tile rows
    auto load_amp = [&](int g, float (&d)[NL], int jl) {
        const float* arow = amp + (size_t)(g * C::RPB + sub) * nx;
#pragma unroll
        for (int r = 0; r < NL; ++r) d[r] = arow[jl + r * T];
    };
    // one buffer each: a group's tile rows are in LDS (and its amplitudes in v's
    // constraint) before the next group's loads into the same registers are issued
    PK cur[K::CPT];
    float acur[NL];
    int g = ir.first;
    if (g >= ir.end) return;  // the whole block (ir is uniform)
    load(g, cur, tid, 0, K::CPT);
    load_amp(g, acur, j);
    for (;;) {
        const bool more = g + ir.step < ir.end;
        // the thread's indices, opaque to the compiler in each iteration: the addresses
        // derived from them are recomputed here instead of being held across the loop
        int jt = j, tt = tid;
        asm volatile("" : "+v"(jt), "+v"(tt));
        lds_barrier();
#pragma unroll
        for (int k = 0; k < K::CPT; ++k) {
            const int c = tt + k * C::THREADS;
#pragma unroll
            for (int e = 0; e < K::CE; ++e) lds[c * K::CE + e] = ST::dec(cur[k].e[e]);
        }
        lds_barrier();
        float2 v[1][E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int x = jt + r * T;
            v[0][r] = lds[(x / kTileW) * C::TS + sub * kTileW + (x % kTileW)];
        }
        lds_barrier();
        // the next group's first PF chunks are loaded during the inverse transform, the rest
        // after the constraint (fewer registers held through the transform)
        if (more) load(g + ir.step, cur, tt, 0, PF);
        const int y0 = g * C::RPB, row = y0 + sub;
        fft<M, E, 1, INV>(v, my_lds, jt, twc);
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            if (r < NL) {
                const float a = acur[r];
                const float re = v[0][r].x * scale, im = v[0][r].y * scale;
                const float m2 = re * re + im * im;
                float2 c;
                if (m2 > 0.f) {
                    const float mag = __fsqrt_rn(m2);
                    const float f = a / mag;
                    c = make_float2(re * f, im * f);
                    const double d = (double)mag - (double)a;
                    acc += d * d;
                } else {
                    c = make_float2(a, 0.f);
                    acc += (double)a * (double)a;
                }
                v[0][r] = c;
            } else {
                v[0][r] = make_float2(0.f, 0.f);
            }
        }
        if (more) load_amp(g + ir.step, acur, jt);
        if constexpr (PF < K::CPT) {
            asm volatile("" ::: "memory");  // these loads stay after the inverse transform
            if (more) load(g + ir.step, cur, tt, PF, K::CPT);
        }
        if (num) row_partials<T>(acc, num, row, jt, true);
        if (out) {
            float2* orow = out + (size_t)row * nx;
#pragma unroll
            for (int r = 0; r < NL; ++r) orow[jt + r * T] = v[0][r];
        } else {
            if (fwd_scale != 1.0f) {
#pragma unroll
                for (int r = 0; r < E; ++r)
                    v[0][r] = make_float2(v[0][r].x * fwd_scale, v[0][r].y * fwd_scale);
            }
            fft_zpad<M, E, 1, FWD>(v, my_lds, jt, twc);
            lds_barrier();
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int x = jt + r * T;
                lds[(x / kTileW) * C::TS + sub * kTileW + (x % kTileW)] = v[0][r];
            }
            lds_barrier();
#pragma unroll
            for (int k = 0; k < K::CPT; ++k) {
                const int c = tt + k * C::THREADS;
                const int t = c / K::PER_TILE, q = c - t * K::PER_TILE;
                PK pk;
#pragma unroll
                for (int e = 0; e < K::CE; ++e) pk.e[e] = ST::enc(lds[c * K::CE + e]);
                *reinterpret_cast<PK*>(spec + ((size_t)t * ny + y0) * kTileW + q * K::CE) = pk;
            }
        }
        if (!more) break;
        g += ir.step;
    }
}

// den = sum(amp^2) in FP64 as kGsDenParts partials, partial b over the contiguous chunk b
// of the array (per-thread strided sums, then a fixed tree): the same order on every run.
__global__ __launch_bounds__(256) void k_gs_den(const float* __restrict__ amp,
                                                double* __restrict__ part, long long count) {
    __shared__ double red[256];
    const long long chunk = (count + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * chunk;
    const long long hi = lo + chunk < count ? lo + chunk : count;
    double t = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += 256) {
        const double a = amp[i];
        t += a * a;
    }
    red[threadIdx.x] = t;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// sum of n values in a fixed order (per-thread strided sums, then a fixed tree); every
// thread of the block gets the result
__device__ double block_sum_fixed(const double* __restrict__ v, int n, double* red) {
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) t += v[i];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// iteration k's error from its n = ny * P row partials and the denominator's partials,
// each summed in a fixed order
__global__ __launch_bounds__(256) void k_gs_errors(const double* __restrict__ num,
                                                   const double* __restrict__ den_part,
                                                   float* __restrict__ errors, int n) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    const double sn = block_sum_fixed(num + (size_t)k * n, n, red);
    const double sd = block_sum_fixed(den_part, kGsDenParts, red);
    if (threadIdx.x == 0) errors[k] = (float)sqrt(sn / sd);
}

// ---- host launchers ------------------------------------------------------------

namespace {
template <class ST>
hipError_t row_gs_t(void* spec, const float* amp, float2* out, double* num, int nx, int ny,
                    int mx, float scale, const float* dyn_inv, float fwd_scale,
                    const float* dyn_fwd, const float2* tw, hipStream_t s, int layout) {
    using SE = typename ST::E;
    const bool half = (mx == 2 * nx);
    if (layout == 1) {
        if (!half) return hipErrorInvalidValue;
        CWO_DISPATCH_M(mx, {
            // (rows of 8192 stay row-major in this loop: no split form of the fused kernel)
            if constexpr (MM >= 2048 && MM <= 4096) {
                // rows of 4096: one row per block, two blocks per CU (6 % faster than two
                // rows per block, measured at 2048^2); rows of 2048: two rows per block
                constexpr int RPB = MM == 4096 ? 1 : 2;
                using C = GsTileCfg<MM, RPB>;
                if (ny % C::RPB != 0) return hipErrorInvalidValue;
                // complex64 rows of 4096: half the next group's chunks in flight during the
                // inverse transform (all of them spilled 28 bytes of registers per lane)
                using K = GsTileChunks<MM, RPB, SE>;
                constexpr int PF = (MM == 4096 && std::is_same_v<ST, StF32>) ? K::CPT / 2 : K::CPT;
                auto k = k_row_gs_tile<MM, ST, RPB, PF>;
                launch_kernel(k, dim3(resident_blocks(k, C::THREADS, ny / C::RPB)),
                                   dim3(C::THREADS), 0, s, (SE*)spec, amp, out, num, nx, ny,
                                   scale, dyn_inv, fwd_scale, dyn_fwd, tw);
            } else {
                return hipErrorInvalidValue;
            }
        });
        return hipGetLastError();
    }
    CWO_DISPATCH_M(mx, {
        using C = RowCfg<MM>;
        dim3 grid((ny + C::RPB - 1) / C::RPB);
        if (half)
            launch_kernel((k_row_gs<MM, true, ST>), grid, dim3(C::THREADS), 0, s, (SE*)spec,
                               amp, out, num, nx, ny, scale, dyn_inv, fwd_scale, dyn_fwd, tw);
        else
            launch_kernel((k_row_gs<MM, false, ST>), grid, dim3(C::THREADS), 0, s, (SE*)spec,
                               amp, out, num, nx, ny, scale, dyn_inv, fwd_scale, dyn_fwd, tw);
    });
    return hipGetLastError();
}
}  // namespace

hipError_t launch_row_gs(void* spec, const float* amp, float2* out, double* num, int nx, int ny,
                         int mx, const GsScale& gsc, const float2* tw, hipStream_t s) {
    switch (gsc.prec) {
        case 0:
            return row_gs_t<StF32>(spec, amp, out, num, nx, ny, mx, gsc.scale, gsc.dyn_inv,
                                   gsc.fwd_scale, gsc.dyn_fwd, tw, s, gsc.layout);
        case 1:
            return row_gs_t<StF16>(spec, amp, out, num, nx, ny, mx, gsc.scale, gsc.dyn_inv,
                                   gsc.fwd_scale, gsc.dyn_fwd, tw, s, gsc.layout);
        case 2:
            return row_gs_t<StBF16>(spec, amp, out, num, nx, ny, mx, gsc.scale, gsc.dyn_inv,
                                    gsc.fwd_scale, gsc.dyn_fwd, tw, s, gsc.layout);
    }
    return hipErrorInvalidValue;
}

int gs_partials(int mx) { return gs_partials_per_row(mx); }

hipError_t launch_gs_errors(const double* num, const float* amp, double* den_work, float* errors,
                            int nx, int ny, int mx, int iters, hipStream_t s) {
    launch_kernel(k_gs_den, dim3(kGsDenParts), dim3(256), 0, s, amp, den_work, (long long)nx * ny);
    launch_kernel(k_gs_errors, dim3(iters), dim3(256), 0, s, num, (const double*)den_work,
                       errors, ny * gs_partials_per_row(mx));
    return hipGetLastError();
}

}  // namespace cwo
