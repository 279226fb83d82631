// Row passes of the padded plane at Mx = 8192 on the tiled layout, in the split form
// (two transforms of half length per row); launched from plane.hip.
#pragma once
#include "column.hpp"

namespace cwo {

// Scaling of the stored planes (powers of two, exact): the field is multiplied by
// sc.in * (*sc.dyn) before the row transform (sc.dyn: a device-computed factor or null).
struct RowScale {
    float in;
    const float* dyn;
};

// ---- row passes of length 2*MH on the tiled plane, as two transforms of length MH -----
//
// With W = exp(-2 pi i/M), M = 2*MH, and a row x_n that is zero for n >= MH, the even bins
// of its length-M transform are DFT_MH(x)[k] and the odd bins DFT_MH(x_n W^n)[k]; the first
// MH values of the length-M inverse transform of a spectrum X are
// IDFT_MH(X_even)[n] + W^-n IDFT_MH(X_odd)[n]. A row is then two length-MH transforms side
// by side (the two-transform exchange of the column pass, 16-byte LDS slots), with one
// LDS exchange fewer than a length-M transform and none of the work on the cropped half.
// W^n for n = j + r*T (T = MH/16 threads per row) is W^j times the constant W_32^r.
// RPB rows per block: a tile row of the group is RPB*kTileW contiguous elements.
template <int MH, int RPB_ = 2>
struct SplitRowCfg {
    static constexpr int E = 16;
    static constexpr int T = MH / E;
    static constexpr int M = 2 * MH;
    static constexpr int RPB = RPB_;
    static constexpr int THREADS = T * RPB;
    static constexpr int TS = kTileW * RPB;              // LDS float2 per tile
    static constexpr int XCH = RPB * 2 * lds_elems<MH>();  // float2: 16-byte slots per row
    static constexpr int TRN = (M / kTileW) * TS;          // regrouping buffer
    static constexpr int LDS = XCH > TRN ? XCH : TRN;
};
template <int MH, int RPB, class SE>
struct SplitChunks {
    using C = SplitRowCfg<MH, RPB>;
    static constexpr int CE = 16 / (int)sizeof(SE);
    static constexpr int PER_TILE = C::RPB * kTileW / CE;
    static constexpr int CPT = (C::M / kTileW) * PER_TILE / C::THREADS;
    static_assert(CPT * C::THREADS == (C::M / kTileW) * PER_TILE, "chunks");
};

// x * W^n for n = j + r*T: wj = W^j, the factor W^(r*T) = W_32^r is a constant of r
template <int DIR, int R>
__device__ __forceinline__ float2 split_twiddle(float2 x, float2 wj) {
    return wconst<32, R, DIR>(ctw<DIR>(x, wj));
}

// Row forward of the split form (persistent, XCD-aware, next group's field values loaded
// while the current group is transformed), spectra regrouped by tile in LDS: thread j holds
// X[2k] and X[2k+1] for k = j + r*T, one 16-byte pair of the same tile row.
template <int MH, int RPB, int PF, bool LATE, class ST, class IN>
__global__ __launch_bounds__((SplitRowCfg<MH, RPB>::THREADS)) __attribute__((amdgpu_waves_per_eu(2))) void k_row_fwd_tsplit(
    IN ins, typename ST::E* __restrict__ out, int nx, int ny, int batch, size_t out_plane,
    RowScale sc, const float2* __restrict__ twm) {
    using C = SplitRowCfg<MH, RPB>;
    constexpr int E = C::E, T = C::T, P = 2;
    using SE = typename ST::E;
    using K = SplitChunks<MH, RPB, SE>;
    using PK = Pack<SE, K::CE>;
    __shared__ float4 lds4[C::LDS / 2];
    float2* lds = reinterpret_cast<float2*>(lds4);
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    const float f = sc.dyn ? sc.in * *sc.dyn : sc.in;
    const int groups = ny * batch / C::RPB;
    const ItemRange ir = xcd_items(blockIdx.x, gridDim.x, groups);
    TwCache<MH, E> twc;
    twc.load(j, twm, 2);
    const float2 wj = twm[j];
    auto load = [&](int g, float2 (&d)[E], int lo, int hi, int jl) {
        const int w = g * C::RPB + sub;  // row of the batch
        const int pl = w / ny, row = w - pl * ny;
        const float2* src = ins(pl) + (size_t)row * nx;
#pragma unroll
        for (int r = lo; r < hi; ++r) d[r] = src[jl + r * T];
    };
    // the next group's first PF values are loaded during the transform, the rest after it
    float2 cur[E];
    int g = ir.first;
    if (g >= ir.end) return;  // the whole block (ir is uniform)
    load(g, cur, 0, E, j);
    // the loop leaves right after the last group, so the prefetch registers are dead
    // during a transform whose successor loads nothing
    for (;;) {
        const bool more = g + ir.step < ir.end;
        // the thread's indices, opaque to the compiler in each iteration: the addresses
        // derived from them are recomputed here instead of being held (or spilled) across
        // the loop
        int jt = j, tt = tid;
        asm volatile("" : "+v"(jt), "+v"(tt));
        float2 v[P][E];
        [&]<int... R>(std::integer_sequence<int, R...>) {
            ((v[0][R] = make_float2(cur[R].x * f, cur[R].y * f),
              v[1][R] = split_twiddle<FWD, R>(v[0][R], wj)), ...);
        }(std::make_integer_sequence<int, E>{});
        if (more) load(g + ir.step, cur, 0, PF, jt);
        fft<MH, E, P, FWD>(v, lds + sub * 2 * lds_elems<MH>(), jt, twc);
        asm volatile("" ::: "memory");  // the remaining loads stay after the transform
        if (more && !LATE) load(g + ir.step, cur, PF, E, jt);
        lds_barrier();
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int k = jt + r * T;  // bins 2k, 2k+1: tile k/2, columns 2(k%2), 2(k%2)+1
            lds4[((k >> 1) * C::TS + sub * kTileW + 2 * (k & 1)) >> 1] =
                make_float4(v[0][r].x, v[0][r].y, v[1][r].x, v[1][r].y);
        }
        lds_barrier();
        const int w0 = g * C::RPB, pl = w0 / ny, y0 = w0 - pl * ny;
        SE* dst = out + pl * out_plane;
#pragma unroll
        for (int k = 0; k < K::CPT; ++k) {
            const int c = tt + k * C::THREADS;
            const int t = c / K::PER_TILE, q = c - t * K::PER_TILE;
            PK pk;
#pragma unroll
            for (int e = 0; e < K::CE; ++e) pk.e[e] = ST::enc(lds[c * K::CE + e]);
            *reinterpret_cast<PK*>(dst + ((size_t)t * ny + y0) * kTileW + q * K::CE) = pk;
        }
        if (!more) break;
        if (LATE) load(g + ir.step, cur, PF, E, jt);
        g += ir.step;
        lds_barrier();
    }
}

// Row inverse of the split form: the mirror of k_row_fwd_tsplit; the output row is
// IDFT(even)[n] + W^-n IDFT(odd)[n], n = j + r*T < MH, scaled.
template <int MH, int RPB, int PF, bool LATE, class OUT, class ST>
__global__ __launch_bounds__((SplitRowCfg<MH, RPB>::THREADS)) __attribute__((amdgpu_waves_per_eu(2))) void k_row_inv_tsplit(
    const typename ST::E* __restrict__ in, OUT outs, int nx, int ny, int batch, size_t in_plane,
    float scale, const float* __restrict__ dyn_inv, const float2* __restrict__ twm) {
    using C = SplitRowCfg<MH, RPB>;
    constexpr int E = C::E, T = C::T, P = 2;
    using SE = typename ST::E;
    using K = SplitChunks<MH, RPB, SE>;
    using PK = Pack<SE, K::CE>;
    __shared__ float4 lds4[C::LDS / 2];
    float2* lds = reinterpret_cast<float2*>(lds4);
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    if (dyn_inv) scale *= *dyn_inv;
    const int groups = ny * batch / C::RPB;
    const ItemRange ir = xcd_items(blockIdx.x, gridDim.x, groups);
    TwCache<MH, E> twc;
    twc.load(j, twm, 2);
    const float2 wj = twm[j];
    auto load = [&](int g, PK (&d)[K::CPT], int lo, int hi, int tl) {
        const int w0 = g * C::RPB, pl = w0 / ny, y0 = w0 - pl * ny;
        const SE* src = in + pl * in_plane;
#pragma unroll
        for (int k = lo; k < hi; ++k) {
            const int c = tl + k * C::THREADS;
            const int t = c / K::PER_TILE, q = c - t * K::PER_TILE;
            d[k] = *reinterpret_cast<const PK*>(src + ((size_t)t * ny + y0) * kTileW + q * K::CE);
        }
    };
    // one buffer: a group's chunks are in LDS before the next group's loads are issued;
    // the first PF chunks are loaded during the transform, the rest after it
    static_assert(PF <= K::CPT, "prefetch");
    PK cur[K::CPT];
    int g = ir.first;
    if (g >= ir.end) return;  // the whole block (ir is uniform)
    load(g, cur, 0, K::CPT, tid);
    for (;;) {
        const bool more = g + ir.step < ir.end;
        // opaque thread indices (see k_row_fwd_tsplit)
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
        float2 v[P][E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int k = jt + r * T;
            const float4 x = lds4[((k >> 1) * C::TS + sub * kTileW + 2 * (k & 1)) >> 1];
            v[0][r] = make_float2(x.x, x.y);
            v[1][r] = make_float2(x.z, x.w);
        }
        lds_barrier();
        if (more) load(g + ir.step, cur, 0, PF, tt);
        fft<MH, E, P, INV>(v, lds + sub * 2 * lds_elems<MH>(), jt, twc);
        asm volatile("" ::: "memory");  // the remaining loads stay after the transform
        if (more && !LATE) load(g + ir.step, cur, PF, K::CPT, tt);
        const int w = g * C::RPB + sub;
        const int pl = w / ny, row = w - pl * ny;
        const size_t base = (size_t)row * nx;
        [&]<int... R>(std::integer_sequence<int, R...>) {
            ((outs.put(pl, base + jt + R * T, [&] {
                 const float2 o = cadd(v[0][R], split_twiddle<INV, R>(v[1][R], wj));
                 return make_float2(o.x * scale, o.y * scale);
             }())), ...);
        }(std::make_integer_sequence<int, E>{});
        if (!more) break;
        if (LATE) {
            asm volatile("" ::: "memory");
            load(g + ir.step, cur, PF, K::CPT, tt);
        }
        g += ir.step;
    }
}

}  // namespace cwo
