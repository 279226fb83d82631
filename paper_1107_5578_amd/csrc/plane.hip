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

#include "column.hpp"

namespace cwo {

// ---- row forward: zero-pad + FFT --------------------------------------------

// Scaling of the stored planes (powers of two, exact): the field is multiplied by
// sc.in * (*sc.dyn) before the row transform (sc.dyn: a device-computed factor or null).
struct RowScale {
    float in;
    const float* dyn;
};

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
    fft<M, E, 1, FWD>(v, lds + sub * lds_elems<M>(), j, twc);
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
        fft<M, E, 1, FWD>(v, lds + sub * lds_elems<M>(), j, twc);
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
    hipLaunchKernelGGL(k_twiddles, dim3((m + 255) / 256), dim3(256), 0, s, tw, m);
    return hipGetLastError();
}

template <class ST, class IN>
static hipError_t launch_row_fwd_t(const IN& ins, void* out, int nx, int ny, int mx, int batch,
                                   size_t out_plane, RowScale sc, const float2* tw,
                                   hipStream_t s, int form = 0) {
    const bool half = (mx == 2 * nx);
    using SE = typename ST::E;
    // persistent form with prefetch where rows are long enough to fill whole blocks
    // (form 2 asks for one row group per block)
    if (half && mx >= 1024 && form != 2) {
        CWO_DISPATCH_M(mx, {
            if constexpr (MM >= 1024) {
                using C = RowCfg<MM>;
                const int groups = (ny * batch + C::RPB - 1) / C::RPB;
                auto k = k_row_fwd_pf<MM, true, ST, IN>;
                hipLaunchKernelGGL(k, dim3(resident_blocks(k, C::THREADS, groups)), dim3(C::THREADS),
                                   0, s, ins, (SE*)out, nx, ny, batch, out_plane, sc, tw);
            }
        });
        return hipGetLastError();
    }
    CWO_DISPATCH_M(mx, {
        using C = RowCfg<MM>;
        dim3 grid((ny + C::RPB - 1) / C::RPB, batch);
        if (half)
            hipLaunchKernelGGL((k_row_fwd<MM, true, ST, IN>), grid, dim3(C::THREADS), 0, s, ins,
                               (SE*)out, nx, ny, out_plane, sc, tw);
        else if constexpr (std::is_same_v<ST, StF32>)
            hipLaunchKernelGGL((k_row_fwd<MM, false, ST, IN>), grid, dim3(C::THREADS), 0, s, ins,
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
        case 0: return launch_row_fwd_t<StF32>(InStrided{in, in_plane}, out, nx, ny, mx, batch, out_plane, sc, tw, s, st.row_form);
        case 1: return launch_row_fwd_t<StF16>(InStrided{in, in_plane}, out, nx, ny, mx, batch, out_plane, sc, tw, s, st.row_form);
        case 2: return launch_row_fwd_t<StBF16>(InStrided{in, in_plane}, out, nx, ny, mx, batch, out_plane, sc, tw, s, st.row_form);
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
                              size_t out_plane, const float2* tw, hipStream_t s) {
    return launch_row_fwd_t<StF32>(ins, out, nx, ny, mx, batch, out_plane,
                                   RowScale{1.0f, nullptr}, tw, s);
}

template <class HF, class ST>
static hipError_t launch_col_t(void* buf, int ny, int my, int mx, int batch, size_t plane,
                               const HF& hf, float hscale, const float2* tw, hipStream_t s) {
    const bool half = (my == 2 * ny);
    using SE = typename ST::E;
    CWO_DISPATCH_M(my, {
        using C = ColCfg<MM>;
        const int items = (mx + C::COLS - 1) / C::COLS * batch;
        if (half) {
            hipLaunchKernelGGL((k_col<MM, true, HF, ST>), dim3(items), dim3(C::THREADS), 0, s,
                               (SE*)buf, ny, mx, batch, plane, hf, hscale, tw);
        } else if constexpr (std::is_same_v<ST, StF32>) {
            hipLaunchKernelGGL((k_col<MM, false, HF, ST>), dim3(items), dim3(C::THREADS), 0, s,
                               (SE*)buf, ny, mx, batch, plane, hf, hscale, tw);
        } else {
            return hipErrorInvalidValue;
        }
    });
    return hipGetLastError();
}

template <class HF>
static hipError_t launch_col_impl(void* buf, int ny, int my, int mx, int batch, size_t plane,
                                  const HF& hf, const Storage& st, const float2* tw,
                                  hipStream_t s) {
    switch (st.prec) {
        case 0: return launch_col_t<HF, StF32>(buf, ny, my, mx, batch, plane, hf, st.col_scale, tw, s);
        case 1: return launch_col_t<HF, StF16>(buf, ny, my, mx, batch, plane, hf, st.col_scale, tw, s);
        case 2: return launch_col_t<HF, StBF16>(buf, ny, my, mx, batch, plane, hf, st.col_scale, tw, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_col_asm(void* buf, int ny, int my, int mx, int batch, size_t plane,
                          const AsmScalars& a, const Storage& st, const float2* tw, hipStream_t s) {
    // largest s = (lambda fx)^2 + (lambda fy)^2 on the grid: the Nyquist corner
    const double sx = a.lam * (0.5 * mx) * a.dfx, sy = a.lam * (0.5 * my) * a.dfy;
    const double smax = sx * sx + sy * sy;
    if (smax <= kAsmFastMaxS) {
        auto fill = [&](auto& hf) {
            hf.lam_dfx = a.lam * a.dfx;
            hf.lam_dfy = a.lam * a.dfy;
            hf.zl = a.zl;
            hf.half_zl = 0.5 * a.zl;
            hf.c0 = (float)(a.zl - std::nearbyint(a.zl));
            hf.mx = mx;
            hf.my = my;
        };
        // the series to s^4 suffices when |zl| times its remainder, at most
        // c_5 smax^5/(1 - smax) with c_5 = 7/256, stays below 2^-28 revolution
        const double s5 = smax * smax * smax * smax * smax;
        if (std::fabs(a.zl) * (7.0 / 256.0) * s5 / (1.0 - smax) <= std::ldexp(1.0, -28)) {
            AsmHFastN<4> hf;
            fill(hf);
            return launch_col_impl(buf, ny, my, mx, batch, plane, hf, st, tw, s);
        }
        AsmHFastN<9> hf;
        fill(hf);
        return launch_col_impl(buf, ny, my, mx, batch, plane, hf, st, tw, s);
    }
    AsmH hf{a.dfx, a.dfy, a.lam, a.zl, mx, my};
    return launch_col_impl(buf, ny, my, mx, batch, plane, hf, st, tw, s);
}

hipError_t launch_col_asm(float2* buf, int ny, int my, int mx, int batch, size_t plane,
                          const AsmScalars& a, const float2* tw, hipStream_t s) {
    return launch_col_asm((void*)buf, ny, my, mx, batch, plane, a, Storage{}, tw, s);
}

hipError_t launch_col_fresnel(void* buf, int ny, int my, int mx, int batch, size_t plane,
                              const float2* hx, const float2* hy, const Storage& st,
                              const float2* tw, hipStream_t s) {
    FresnelH hf{hx, hy};
    return launch_col_impl(buf, ny, my, mx, batch, plane, hf, st, tw, s);
}

template <class OUT, class ST>
static hipError_t launch_row_inv_t(const void* in, const OUT& outs, int nx, int ny, int mx,
                                   int batch, size_t in_plane, float scale, const float* dyn_inv,
                                   const float2* tw, hipStream_t s, int form = 0) {
    const bool half = (mx == 2 * nx);
    using SE = typename ST::E;
    if (half && mx >= 1024 && form != 2) {
        CWO_DISPATCH_M(mx, {
            if constexpr (MM >= 1024) {
                using C = RowCfg<MM>;
                const int groups = (ny * batch + C::RPB - 1) / C::RPB;
                auto k = k_row_inv_pf<MM, true, OUT, ST>;
                hipLaunchKernelGGL(k, dim3(resident_blocks(k, C::THREADS, groups)), dim3(C::THREADS),
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
            hipLaunchKernelGGL((k_row_inv<MM, true, OUT, ST>), grid, dim3(C::THREADS), 0, s,
                               (const SE*)in, outs, nx, ny, in_plane, scale, dyn_inv, tw);
        else if constexpr (std::is_same_v<ST, StF32>)
            hipLaunchKernelGGL((k_row_inv<MM, false, OUT, ST>), grid, dim3(C::THREADS), 0, s,
                               (const SE*)in, outs, nx, ny, in_plane, scale, dyn_inv, tw);
        else
            return hipErrorInvalidValue;
    });
    return hipGetLastError();
}

template <class OUT>
static hipError_t launch_row_inv_impl(const float2* in, const OUT& outs, int nx, int ny, int mx,
                                      int batch, size_t in_plane, float scale, const float2* tw,
                                      hipStream_t s) {
    return launch_row_inv_t<OUT, StF32>(in, outs, nx, ny, mx, batch, in_plane, scale, nullptr, tw,
                                        s);
}

hipError_t launch_row_inv(const float2* in, float2* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, float scale, const float2* tw,
                          hipStream_t s) {
    return launch_row_inv_impl(in, OutStrided{out, out_plane}, nx, ny, mx, batch, in_plane, scale,
                               tw, s);
}

hipError_t launch_row_inv_tab(const float2* in, const OutTable& outs, int nx, int ny, int mx,
                              int batch, size_t in_plane, float scale, const float2* tw,
                              hipStream_t s) {
    return launch_row_inv_impl(in, outs, nx, ny, mx, batch, in_plane, scale, tw, s);
}

hipError_t launch_row_inv_intensity(const void* in, float* out, int nx, int ny, int mx,
                                    const Storage& st, const float2* tw, hipStream_t s) {
    const OutIntensity o{out, 0};
    switch (st.prec) {
        case 0:
            return launch_row_inv_t<OutIntensity, StF32>(in, o, nx, ny, mx, 1, 0, st.out_scale,
                                                         st.dyn_inv, tw, s, st.row_form);
        case 1:
            return launch_row_inv_t<OutIntensity, StF16>(in, o, nx, ny, mx, 1, 0, st.out_scale,
                                                         st.dyn_inv, tw, s, st.row_form);
        case 2:
            return launch_row_inv_t<OutIntensity, StBF16>(in, o, nx, ny, mx, 1, 0, st.out_scale,
                                                          st.dyn_inv, tw, s, st.row_form);
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
                                                       st.row_form);
        case 1:
            return launch_row_inv_t<OutStrided, StF16>(in, o, nx, ny, mx, batch, in_plane,
                                                       st.out_scale, st.dyn_inv, tw, s,
                                                       st.row_form);
        case 2:
            return launch_row_inv_t<OutStrided, StBF16>(in, o, nx, ny, mx, batch, in_plane,
                                                        st.out_scale, st.dyn_inv, tw, s,
                                                       st.row_form);
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
    hipLaunchKernelGGL((k_absmax_partial<T>), dim3(nb), dim3(256), 0, s, in, n, work + 2);
    hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(256), 0, s, (const float*)(work + 2), nb, work);
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
