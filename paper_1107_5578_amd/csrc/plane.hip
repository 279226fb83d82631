// HIP kernels of the diffraction hot path (gfx950).
//
// One propagation of an Ny x Nx complex64 field through the 2Ny x 2Nx padded
// convolution of the paper's convolution-form diffractions (Sec. 2.1.6) is
// three kernels on a [Ny][Mx] complex64 scratch plane:
//
//   row_fwd : for each of the Ny field rows, load Nx values (the Mx - Nx pad
//             values are implicit zeros), forward FFT of length Mx, store the
//             spectrum row. Rows Ny..My-1 of the padded grid are all zero and
//             are never materialised.
//   col     : for each of the Mx columns, load its Ny non-zero rows, forward
//             FFT of length My, multiply by the transfer function of the bin
//             (generated in the kernel), inverse FFT of length My, store the
//             first Ny rows back in place (the crop along y).
//   row_inv : for each of the Ny rows, inverse FFT of length Mx, keep the
//             first Nx values, scale by 1/(Mx*My) and store the output.
//
// Transfer functions (the multiply step of Eqs. ang3 and fre_conv_fft):
//   ASM     : H = exp(i*z*k*sqrt(1 - s)), s = (lambda fx)^2 + (lambda fy)^2,
//             H = 0 for s > 1; the phase in revolutions t = (z/lambda)sqrt(1-s)
//             and its reduction t - rint(t) are FP64, the sine/cosine FP32.
//   Fresnel : H = C * Hx[p] * Hy[q]; the FFT of the sampled impulse response
//             h_F factorises into two 1-D transforms of chirps, computed here
//             by FP64 FFTs.

#include "rowsplit.hpp"

namespace cwo {

// ---- row forward: zero-pad + FFT --------------------------------------------

template <int M, bool HALF, class ST, class IN>
__global__ __launch_bounds__(RowCfg<M>::THREADS) void k_row_fwd(IN ins,
                                                                  typename ST::E* __restrict__ out,
                                                                  int nx, int ny, size_t out_plane,
                                                                  RowScale sc,
                                                                  const float2* __restrict__ tw) {
    using C = RowCfg<M>;
    constexpr int E = C::E, T = C::T;
    const float f = sc.dyn ? sc.in * *sc.dyn : sc.in;
    __shared__ float2 lds[C::RPB * lds_elems<M>()];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    const int row = blockIdx.x * C::RPB + sub;
    const bool valid = row < ny;
    const float2* src = ins(blockIdx.y) + (size_t)(valid ? row : 0) * nx;
    TwCache<M, E> twc;
    twc.load(j, tw);
    float2 v[1][E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = j + r * T;
        if constexpr (HALF) {
            // M == 2*nx: exactly the first E/2 registers hold field values
            v[0][r] = (r < E / 2 && valid) ? src[x] : make_float2(0.f, 0.f);
        } else {
            v[0][r] = (valid && x < nx) ? src[x] : make_float2(0.f, 0.f);
        }
    }
    if (f != 1.0f) {
#pragma unroll
        for (int r = 0; r < E; ++r) v[0][r] = make_float2(v[0][r].x * f, v[0][r].y * f);
    }
    if constexpr (HALF) fft_zpad<M, E, 1, FWD>(v, lds + sub * lds_elems<M>(), j, twc);
    else fft<M, E, 1, FWD>(v, lds + sub * lds_elems<M>(), j, twc);
    if (valid) {
        typename ST::E* dst = out + blockIdx.y * out_plane + (size_t)row * M;
#pragma unroll
        for (int r = 0; r < E; ++r) dst[j + r * T] = ST::enc(v[0][r]);
    }
}

// Persistent form: a grid of resident blocks walks the rows (block b takes row groups
// b, b + G, ...) and issues the next group's loads before transforming the current one.
template <int M, bool HALF, class ST, class IN>
__global__ __launch_bounds__(RowCfg<M>::THREADS) void k_row_fwd_pf(IN ins,
                                                                     typename ST::E* __restrict__ out,
                                                                     int nx, int ny, int batch,
                                                                     size_t out_plane, RowScale sc,
                                                                     const float2* __restrict__ tw) {
    using C = RowCfg<M>;
    constexpr int E = C::E, T = C::T;
    constexpr int NL = HALF ? E / 2 : E;
    __shared__ float2 lds[C::RPB * lds_elems<M>()];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    const float f = sc.dyn ? sc.in * *sc.dyn : sc.in;
    const int rows = ny * batch;
    const int groups = (rows + C::RPB - 1) / C::RPB;
    TwCache<M, E> twc;
    twc.load(j, tw);
    auto load = [&](int g, float2 (&d)[NL]) {
        const int w = g * C::RPB + sub;
        const bool ok = w < rows;
        const int pl = ok ? w / ny : 0, row = ok ? w - pl * ny : 0;
        const float2* src = ins(pl) + (size_t)row * nx;
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int x = j + r * T;
            d[r] = (ok && (HALF || x < nx)) ? src[x] : make_float2(0.f, 0.f);
        }
    };
    float2 cur[NL], nxt[NL];
    int g = blockIdx.x;
    if (g < groups) load(g, cur);
    for (; g < groups; g += gridDim.x) {
        if (g + (int)gridDim.x < groups) load(g + gridDim.x, nxt);
        float2 v[1][E];
#pragma unroll
        for (int r = 0; r < E; ++r)
            v[0][r] = r < NL ? make_float2(cur[r].x * f, cur[r].y * f) : make_float2(0.f, 0.f);
        if constexpr (HALF) fft_zpad<M, E, 1, FWD>(v, lds + sub * lds_elems<M>(), j, twc);
        else fft<M, E, 1, FWD>(v, lds + sub * lds_elems<M>(), j, twc);
        const int w = g * C::RPB + sub;
        if (w < rows) {
            const int pl = w / ny, row = w - pl * ny;
            typename ST::E* dst = out + pl * out_plane + (size_t)row * M;
#pragma unroll
            for (int r = 0; r < E; ++r) dst[j + r * T] = ST::enc(v[0][r]);
        }
#pragma unroll
        for (int r = 0; r < NL; ++r) cur[r] = nxt[r];
    }
}

// ---- row inverse: IFFT + crop + normalisation ---------------------------------

template <int M, bool HALF, class OUT, class ST>
__global__ __launch_bounds__(RowCfg<M>::THREADS) void k_row_inv(
    const typename ST::E* __restrict__ in, OUT outs, int nx, int ny, size_t in_plane, float scale,
    const float* __restrict__ dyn_inv, const float2* __restrict__ tw) {
    using C = RowCfg<M>;
    constexpr int E = C::E, T = C::T;
    if (dyn_inv) scale *= *dyn_inv;
    __shared__ float2 lds[C::RPB * lds_elems<M>()];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    const int row = blockIdx.x * C::RPB + sub;
    const bool valid = row < ny;
    const typename ST::E* src = in + blockIdx.y * in_plane + (size_t)(valid ? row : 0) * M;
    TwCache<M, E> twc;
    twc.load(j, tw);
    float2 v[1][E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[0][r] = valid ? ST::dec(src[j + r * T]) : make_float2(0.f, 0.f);
    fft<M, E, 1, INV>(v, lds + sub * lds_elems<M>(), j, twc);
    if (valid) {
        const size_t base = (size_t)row * nx;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int x = j + r * T;
            const float2 o = make_float2(v[0][r].x * scale, v[0][r].y * scale);
            if constexpr (HALF) {
                if (r < E / 2) outs.put(blockIdx.y, base + x, o);
            } else {
                if (x < nx) outs.put(blockIdx.y, base + x, o);
            }
        }
    }
}

// Persistent form of the row inverse (see k_row_fwd_pf).
template <int M, bool HALF, class OUT, class ST>
__global__ __launch_bounds__(RowCfg<M>::THREADS) void k_row_inv_pf(
    const typename ST::E* __restrict__ in, OUT outs, int nx, int ny, int batch, size_t in_plane,
    float scale, const float* __restrict__ dyn_inv, const float2* __restrict__ tw) {
    using C = RowCfg<M>;
    constexpr int E = C::E, T = C::T;
    __shared__ float2 lds[C::RPB * lds_elems<M>()];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    if (dyn_inv) scale *= *dyn_inv;
    const int rows = ny * batch;
    const int groups = (rows + C::RPB - 1) / C::RPB;
    TwCache<M, E> twc;
    twc.load(j, tw);
    using SE = typename ST::E;
    auto load = [&](int g, SE (&d)[E]) {
        const int w = g * C::RPB + sub;
        const bool ok = w < rows;
        const int pl = ok ? w / ny : 0, row = ok ? w - pl * ny : 0;
        const SE* src = in + pl * in_plane + (size_t)row * M;
#pragma unroll
        for (int r = 0; r < E; ++r) d[r] = src[j + r * T];
    };
    SE cur[E], nxt[E];
    int g = blockIdx.x;
    if (g < groups) load(g, cur);
    for (; g < groups; g += gridDim.x) {
        if (g + (int)gridDim.x < groups) load(g + gridDim.x, nxt);
        float2 v[1][E];
#pragma unroll
        for (int r = 0; r < E; ++r) v[0][r] = ST::dec(cur[r]);
        fft<M, E, 1, INV>(v, lds + sub * lds_elems<M>(), j, twc);
        const int w = g * C::RPB + sub;
        if (w < rows) {
            const int pl = w / ny, row = w - pl * ny;
            const size_t base = (size_t)row * nx;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int x = j + r * T;
                if (HALF ? (r < E / 2) : (x < nx))
                    outs.put(pl, base + x, make_float2(v[0][r].x * scale, v[0][r].y * scale));
            }
        }
#pragma unroll
        for (int r = 0; r < E; ++r) cur[r] = nxt[r];
    }
}

// ---- row passes on the tiled plane ----------------------------------------------

// Row forward into the tiled plane (padded rows, Mx = 2Nx). A resident grid walks groups
// of RPB consecutive rows of the batch (the blocks of one XCD take that XCD's contiguous
// range of groups, so the rows that share a tile line are written through one L2); the
// next group's field values are loaded into registers while the current group is
// transformed. The RPB row spectra are then regrouped in LDS by tile, and each thread
// stores whole tile rows: RPB*kTileW contiguous elements per tile and group.
template <int M, class ST, class IN>
__global__ __launch_bounds__(TileRowCfg<M>::THREADS) void k_row_fwd_tile(
    IN ins, typename ST::E* __restrict__ out, int nx, int ny, int batch, size_t out_plane,
    RowScale sc, const float2* __restrict__ tw) {
    using C = TileRowCfg<M>;
    constexpr int E = C::E, T = C::T, NL = E / 2;
    using SE = typename ST::E;
    using K = TileChunks<M, SE>;
    using PK = Pack<SE, K::CE>;
    __shared__ float2 lds[C::LDS];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    const float f = sc.dyn ? sc.in * *sc.dyn : sc.in;
    const int groups = ny * batch / C::RPB;
    const ItemRange ir = xcd_items(blockIdx.x, gridDim.x, groups);
    TwCache<M, E> twc;
    twc.load(j, tw);
    auto load = [&](int g, float2 (&d)[NL]) {
        const int w = g * C::RPB + sub;  // row of the batch
        const int pl = w / ny, row = w - pl * ny;
        const float2* src = ins(pl) + (size_t)row * nx;
#pragma unroll
        for (int r = 0; r < NL; ++r) d[r] = src[j + r * T];
    };
    float2 cur[NL], nxt[NL];
    int g = ir.first;
    if (g < ir.end) load(g, cur);
    for (; g < ir.end; g += ir.step) {
        if (g + ir.step < ir.end) load(g + ir.step, nxt);
        float2 v[1][E];
#pragma unroll
        for (int r = 0; r < E; ++r)
            v[0][r] = r < NL ? make_float2(cur[r].x * f, cur[r].y * f) : make_float2(0.f, 0.f);
        fft_zpad<M, E, 1, FWD>(v, lds + sub * lds_elems<M>(), j, twc);
        // regroup by tile (the barriers also keep the compiler from moving LDS accesses
        // across the phases)
        lds_barrier();
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int x = j + r * T;
            lds[(x / kTileW) * C::TS + sub * kTileW + (x % kTileW)] = v[0][r];
        }
        lds_barrier();
        const int w0 = g * C::RPB, pl = w0 / ny, y0 = w0 - pl * ny;
        SE* dst = out + pl * out_plane;
#pragma unroll
        for (int k = 0; k < K::CPT; ++k) {
            const int c = tid + k * C::THREADS;
            const int t = c / K::PER_TILE, q = c - t * K::PER_TILE;
            PK pk;
#pragma unroll
            for (int e = 0; e < K::CE; ++e) pk.e[e] = ST::enc(lds[c * K::CE + e]);
            *reinterpret_cast<PK*>(dst + ((size_t)t * ny + y0) * kTileW + q * K::CE) = pk;
        }
        lds_barrier();
#pragma unroll
        for (int r = 0; r < NL; ++r) cur[r] = nxt[r];
    }
}

// Row inverse from the tiled plane: the mirror of k_row_fwd_tile. Each thread loads
// whole tile rows of the next group while the current one is transformed; a group's
// tile rows are regrouped in LDS into rows, transformed, cropped to the first Nx values
// and scaled.
template <int M, class OUT, class ST>
__global__ __launch_bounds__(TileRowCfg<M>::THREADS) void k_row_inv_tile(
    const typename ST::E* __restrict__ in, OUT outs, int nx, int ny, int batch, size_t in_plane,
    float scale, const float* __restrict__ dyn_inv, const float2* __restrict__ tw) {
    using C = TileRowCfg<M>;
    constexpr int E = C::E, T = C::T;
    using SE = typename ST::E;
    using K = TileChunks<M, SE>;
    using PK = Pack<SE, K::CE>;
    __shared__ float2 lds[C::LDS];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    if (dyn_inv) scale *= *dyn_inv;
    const int groups = ny * batch / C::RPB;
    const ItemRange ir = xcd_items(blockIdx.x, gridDim.x, groups);
    TwCache<M, E> twc;
    twc.load(j, tw);
    auto load = [&](int g, PK (&d)[K::CPT]) {
        const int w0 = g * C::RPB, pl = w0 / ny, y0 = w0 - pl * ny;
        const SE* src = in + pl * in_plane;
#pragma unroll
        for (int k = 0; k < K::CPT; ++k) {
            const int c = tid + k * C::THREADS;
            const int t = c / K::PER_TILE, q = c - t * K::PER_TILE;
            d[k] = *reinterpret_cast<const PK*>(src + ((size_t)t * ny + y0) * kTileW + q * K::CE);
        }
    };
    PK cur[K::CPT], nxt[K::CPT];
    int g = ir.first;
    if (g < ir.end) load(g, cur);
    for (; g < ir.end; g += ir.step) {
        lds_barrier();
#pragma unroll
        for (int k = 0; k < K::CPT; ++k) {
            const int c = tid + k * C::THREADS;
#pragma unroll
            for (int e = 0; e < K::CE; ++e) lds[c * K::CE + e] = ST::dec(cur[k].e[e]);
        }
        lds_barrier();
        float2 v[1][E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int x = j + r * T;
            v[0][r] = lds[(x / kTileW) * C::TS + sub * kTileW + (x % kTileW)];
        }
        lds_barrier();
        if (g + ir.step < ir.end) load(g + ir.step, nxt);
        fft<M, E, 1, INV>(v, lds + sub * lds_elems<M>(), j, twc);
        const int w = g * C::RPB + sub;
        const int pl = w / ny, row = w - pl * ny;
        const size_t base = (size_t)row * nx;
#pragma unroll
        for (int r = 0; r < E / 2; ++r)
            outs.put(pl, base + j + r * T, make_float2(v[0][r].x * scale, v[0][r].y * scale));
#pragma unroll
        for (int k = 0; k < K::CPT; ++k) cur[k] = nxt[k];
    }
}

// ---- tables -------------------------------------------------------------------

// tw[k] = exp(-2*pi*i*k/M), evaluated in FP64 and rounded once to FP32
__global__ void k_twiddles(float2* tw, int m) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    double s, c;
    sincospi(2.0 * (double)k / (double)m, &s, &c);
    tw[k] = make_float2((float)c, (float)(-s));
}

// ---- host launchers ------------------------------------------------------------

hipError_t launch_twiddles(float2* tw, int m, hipStream_t s) {
    launch_kernel(k_twiddles, dim3((m + 255) / 256), dim3(256), 0, s, tw, m);
    return hipGetLastError();
}

template <class ST, class IN>
static hipError_t launch_row_fwd_t(const IN& ins, void* out, int nx, int ny, int mx, int batch,
                                   size_t out_plane, RowScale sc, const float2* tw,
                                   hipStream_t s, int form = 0, int layout = 0) {
    const bool half = (mx == 2 * nx);
    using SE = typename ST::E;
    if (layout == 1) {
        if (!half) return hipErrorInvalidValue;
        CWO_DISPATCH_M(mx, {
            if constexpr (MM == 8192) {
                // two rows per block, the next group's values all loaded during the transform
                using C = SplitRowCfg<MM / 2, 2>;
                if ((ny * batch) % C::RPB != 0) return hipErrorInvalidValue;
                const int groups = ny * batch / C::RPB;
                auto k = k_row_fwd_tsplit<MM / 2, 2, C::E, false, ST, IN>;
                launch_kernel(k, dim3(resident_blocks(k, C::THREADS, groups)), dim3(C::THREADS),
                                   0, s, ins, (SE*)out, nx, ny, batch, out_plane, sc, tw);
            } else if constexpr (MM >= 2048) {
                using C = TileRowCfg<MM>;
                const int groups = ny * batch / C::RPB;
                auto k = k_row_fwd_tile<MM, ST, IN>;
                launch_kernel(k, dim3(resident_blocks(k, C::THREADS, groups)), dim3(C::THREADS),
                                   0, s, ins, (SE*)out, nx, ny, batch, out_plane, sc, tw);
            } else {
                return hipErrorInvalidValue;
            }
        });
        return hipGetLastError();
    }
    // persistent form with prefetch where rows are long enough to fill whole blocks
    // (form 2 asks for one row group per block)
    if (half && mx >= 1024 && form != 2) {
        CWO_DISPATCH_M(mx, {
            if constexpr (MM >= 1024) {
                using C = RowCfg<MM>;
                const int groups = (ny * batch + C::RPB - 1) / C::RPB;
                auto k = k_row_fwd_pf<MM, true, ST, IN>;
                launch_kernel(k, dim3(resident_blocks(k, C::THREADS, groups)), dim3(C::THREADS),
                                   0, s, ins, (SE*)out, nx, ny, batch, out_plane, sc, tw);
            }
        });
        return hipGetLastError();
    }
    CWO_DISPATCH_M(mx, {
        using C = RowCfg<MM>;
        dim3 grid((ny + C::RPB - 1) / C::RPB, batch);
        if (half)
            launch_kernel((k_row_fwd<MM, true, ST, IN>), grid, dim3(C::THREADS), 0, s, ins,
                               (SE*)out, nx, ny, out_plane, sc, tw);
        else if constexpr (std::is_same_v<ST, StF32>)
            launch_kernel((k_row_fwd<MM, false, ST, IN>), grid, dim3(C::THREADS), 0, s, ins,
                               (SE*)out, nx, ny, out_plane, sc, tw);
        else
            return hipErrorInvalidValue;
    });
    return hipGetLastError();
}

hipError_t launch_row_fwd(const float2* in, void* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, const Storage& st, const float2* tw,
                          hipStream_t s) {
    const RowScale sc{st.in_scale, st.dyn_scale};
    switch (st.prec) {
        case 0: return launch_row_fwd_t<StF32>(InStrided{in, in_plane}, out, nx, ny, mx, batch, out_plane, sc, tw, s, st.row_form, st.layout);
        case 1: return launch_row_fwd_t<StF16>(InStrided{in, in_plane}, out, nx, ny, mx, batch, out_plane, sc, tw, s, st.row_form, st.layout);
        case 2: return launch_row_fwd_t<StBF16>(InStrided{in, in_plane}, out, nx, ny, mx, batch, out_plane, sc, tw, s, st.row_form, st.layout);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_row_fwd(const float2* in, float2* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, const float2* tw, hipStream_t s,
                          int row_form) {
    return launch_row_fwd_t<StF32>(InStrided{in, in_plane}, out, nx, ny, mx, batch, out_plane,
                                   RowScale{1.0f, nullptr}, tw, s, row_form);
}

hipError_t launch_row_fwd_tab(const InTable& ins, float2* out, int nx, int ny, int mx, int batch,
                              size_t out_plane, const float2* tw, hipStream_t s, int layout) {
    return launch_row_fwd_t<StF32>(ins, out, nx, ny, mx, batch, out_plane,
                                   RowScale{1.0f, nullptr}, tw, s, 0, layout);
}

template <class OUT, class ST>
static hipError_t launch_row_inv_t(const void* in, const OUT& outs, int nx, int ny, int mx,
                                   int batch, size_t in_plane, float scale, const float* dyn_inv,
                                   const float2* tw, hipStream_t s, int form = 0,
                                   int layout = 0) {
    const bool half = (mx == 2 * nx);
    using SE = typename ST::E;
    if (layout == 1) {
        if (!half) return hipErrorInvalidValue;
        CWO_DISPATCH_M(mx, {
            if constexpr (MM == 8192) {
                // complex64: two rows per block, 8 of the next group's 16 chunks loaded
                // during the transform; 16-bit storage: one row per block (two blocks per
                // CU), 4 of 8 chunks during the transform and the rest after the stores
                // (measured at 4096^2)
                constexpr bool F32 = std::is_same_v<ST, StF32>;
                constexpr int RPB = F32 ? 2 : 1, PF = F32 ? 8 : 4;
                using C = SplitRowCfg<MM / 2, RPB>;
                if ((ny * batch) % C::RPB != 0) return hipErrorInvalidValue;
                const int groups = ny * batch / C::RPB;
                auto k = k_row_inv_tsplit<MM / 2, RPB, PF, !F32, OUT, ST>;
                launch_kernel(k, dim3(resident_blocks(k, C::THREADS, groups)), dim3(C::THREADS),
                                   0, s, (const SE*)in, outs, nx, ny, batch, in_plane, scale,
                                   dyn_inv, tw);
            } else if constexpr (MM >= 2048) {
                using C = TileRowCfg<MM>;
                const int groups = ny * batch / C::RPB;
                auto k = k_row_inv_tile<MM, OUT, ST>;
                launch_kernel(k, dim3(resident_blocks(k, C::THREADS, groups)), dim3(C::THREADS),
                                   0, s, (const SE*)in, outs, nx, ny, batch, in_plane, scale,
                                   dyn_inv, tw);
            } else {
                return hipErrorInvalidValue;
            }
        });
        return hipGetLastError();
    }
    if (half && mx >= 1024 && form != 2) {
        CWO_DISPATCH_M(mx, {
            if constexpr (MM >= 1024) {
                using C = RowCfg<MM>;
                const int groups = (ny * batch + C::RPB - 1) / C::RPB;
                auto k = k_row_inv_pf<MM, true, OUT, ST>;
                launch_kernel(k, dim3(resident_blocks(k, C::THREADS, groups)), dim3(C::THREADS),
                                   0, s, (const SE*)in, outs, nx, ny, batch, in_plane, scale,
                                   dyn_inv, tw);
            }
        });
        return hipGetLastError();
    }
    CWO_DISPATCH_M(mx, {
        using C = RowCfg<MM>;
        dim3 grid((ny + C::RPB - 1) / C::RPB, batch);
        if (half)
            launch_kernel((k_row_inv<MM, true, OUT, ST>), grid, dim3(C::THREADS), 0, s,
                               (const SE*)in, outs, nx, ny, in_plane, scale, dyn_inv, tw);
        else if constexpr (std::is_same_v<ST, StF32>)
            launch_kernel((k_row_inv<MM, false, OUT, ST>), grid, dim3(C::THREADS), 0, s,
                               (const SE*)in, outs, nx, ny, in_plane, scale, dyn_inv, tw);
        else
            return hipErrorInvalidValue;
    });
    return hipGetLastError();
}

template <class OUT>
static hipError_t launch_row_inv_impl(const float2* in, const OUT& outs, int nx, int ny, int mx,
                                      int batch, size_t in_plane, float scale, const float2* tw,
                                      hipStream_t s, int layout = 0) {
    return launch_row_inv_t<OUT, StF32>(in, outs, nx, ny, mx, batch, in_plane, scale, nullptr, tw,
                                        s, 0, layout);
}

hipError_t launch_row_inv(const float2* in, float2* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, float scale, const float2* tw,
                          hipStream_t s) {
    return launch_row_inv_impl(in, OutStrided{out, out_plane}, nx, ny, mx, batch, in_plane, scale,
                               tw, s);
}

hipError_t launch_row_inv_tab(const float2* in, const OutTable& outs, int nx, int ny, int mx,
                              int batch, size_t in_plane, float scale, const float2* tw,
                              hipStream_t s, int layout) {
    return launch_row_inv_impl(in, outs, nx, ny, mx, batch, in_plane, scale, tw, s, layout);
}

hipError_t launch_row_inv_intensity(const void* in, float* out, int nx, int ny, int mx,
                                    const Storage& st, const float2* tw, hipStream_t s) {
    const OutIntensity o{out, 0};
    switch (st.prec) {
        case 0:
            return launch_row_inv_t<OutIntensity, StF32>(in, o, nx, ny, mx, 1, 0, st.out_scale,
                                                         st.dyn_inv, tw, s, st.row_form, st.layout);
        case 1:
            return launch_row_inv_t<OutIntensity, StF16>(in, o, nx, ny, mx, 1, 0, st.out_scale,
                                                         st.dyn_inv, tw, s, st.row_form, st.layout);
        case 2:
            return launch_row_inv_t<OutIntensity, StBF16>(in, o, nx, ny, mx, 1, 0, st.out_scale,
                                                          st.dyn_inv, tw, s, st.row_form, st.layout);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_row_inv(const void* in, float2* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, const Storage& st, const float2* tw,
                          hipStream_t s) {
    const OutStrided o{out, out_plane};
    switch (st.prec) {
        case 0:
            return launch_row_inv_t<OutStrided, StF32>(in, o, nx, ny, mx, batch, in_plane,
                                                       st.out_scale, st.dyn_inv, tw, s,
                                                       st.row_form, st.layout);
        case 1:
            return launch_row_inv_t<OutStrided, StF16>(in, o, nx, ny, mx, batch, in_plane,
                                                       st.out_scale, st.dyn_inv, tw, s,
                                                       st.row_form, st.layout);
        case 2:
            return launch_row_inv_t<OutStrided, StBF16>(in, o, nx, ny, mx, batch, in_plane,
                                                        st.out_scale, st.dyn_inv, tw, s,
                                                        st.row_form, st.layout);
    }
    return hipErrorInvalidValue;
}

// ---- range of a field for FP16 storage -----------------------------------------

__device__ __forceinline__ float absmax(float2 v) { return fmaxf(fabsf(v.x), fabsf(v.y)); }
__device__ __forceinline__ float absmax(float v) { return fabsf(v); }

// per-block maximum of |re|, |im| (of |a| for a real array) over a grid-strided range
template <class T>
__global__ __launch_bounds__(256) void k_absmax_partial(const T* __restrict__ in, size_t n,
                                                        float* __restrict__ partial) {
    __shared__ float red[256];
    float m = 0.f;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        m = fmaxf(m, absmax(in[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// scale[0] = 2^-e with e = ceil(log2(max)) (so the scaled field is within [-1, 1]),
// scale[1] = 2^e; both 1 when the field is zero or not finite
__global__ __launch_bounds__(256) void k_absmax_final(const float* __restrict__ partial, int np,
                                                      float* __restrict__ scale) {
    __shared__ float red[256];
    float m = 0.f;
    for (int i = threadIdx.x; i < np; i += 256) m = fmaxf(m, partial[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float mx = red[0];
        int e = 0;
        if (mx > 0.f && isfinite(mx)) {
            const float f = frexpf(mx, &e);  // mx = f * 2^e, f in [0.5, 1)
            (void)f;
        }
        scale[0] = ldexpf(1.0f, -e);
        scale[1] = ldexpf(1.0f, e);
    }
}

namespace {
template <class T>
hipError_t range_scale_t(const T* in, size_t n, float* work, hipStream_t s) {
    const size_t want = (n + 256 * 16 - 1) / (256 * 16);
    const int nb = want < 1 ? 1 : (want < (size_t)kRangeBlocks ? (int)want : kRangeBlocks);
    launch_kernel((k_absmax_partial<T>), dim3(nb), dim3(256), 0, s, in, n, work + 2);
    launch_kernel(k_absmax_final, dim3(1), dim3(256), 0, s, (const float*)(work + 2), nb, work);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_range_scale(const float2* in, size_t n, float* work, hipStream_t s) {
    return range_scale_t(in, n, work, s);
}

hipError_t launch_range_scale(const float* in, size_t n, float* work, hipStream_t s) {
    return range_scale_t(in, n, work, s);
}

}  // namespace cwo
