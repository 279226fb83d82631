// Column pass of the diffraction path: forward FFT along y, multiplication by the
// transfer function generated per bin, inverse FFT, crop (shared by the plain, shifted
// and ping-pong forms).
#pragma once
#include "kernel_common.hpp"

namespace cwo {

// ---- column pass: FFT, transfer function, IFFT, crop --------------------------

// Exact form, for any parameters: per bin in FP64, the propagating test s <= 1 evaluated
// as lam*(p'*df) squared and summed, each operation rounded on its own (fused
// multiply-adds are switched off, so the decision is that of the plain FP64 definition),
// sine/cosine of the reduced phase in FP32.
struct AsmH {
    double dfx, dfy;  // frequency pitches 1/(Mx dx), 1/(My dy)
    double lam;       // wavelength
    double zl;        // z / lambda: phase in revolutions per unit sqrt(1 - s)
    int mx, my;
    struct Col {
        double ax2;
    };
    __device__ __forceinline__ Col column(int p) const {
#pragma clang fp contract(off)
        const double pp = (double)(p < mx / 2 ? p : p - mx);
        const double ax = lam * (pp * dfx);
        return Col{ax * ax};
    }
    struct Row {
        double ay2;
    };
    __device__ __forceinline__ Row row(int q) const {
#pragma clang fp contract(off)
        const double qq = (double)(q < my / 2 ? q : q - my);
        const double ay = lam * (qq * dfy);
        return Row{ay * ay};
    }
    __device__ __forceinline__ float2 operator()(const Col& c, const Row& rw) const {
#pragma clang fp contract(off)
        // s = (lambda*fx)^2 + (lambda*fy)^2 with fx = p'*dfx, evaluated without contraction
        const double s = rw.ay2 + c.ax2;
        if (!(s <= 1.0)) return make_float2(0.f, 0.f);  // evanescent bin
        const double t = zl * sqrt(1.0 - s);             // revolutions
        const float r = (float)(t - rint(t));            // [-0.5, 0.5]
        return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
    }
};

// Fast form, used when every bin has s <= 0.05 (so none is evanescent). With
// T(s) = 1 - s/2 - sqrt(1 - s), the phase in revolutions splits exactly into
//     (z/lambda) sqrt(1 - s) = zl - zl*a/2 - zl*b/2 - zl*T(s),  s = a + b,
// a = (lambda fx)^2 per column, b = (lambda fy)^2 per row. Every large term is
// reduced modulo one revolution in FP64 before it is rounded to FP32; T(s) is the
// power series sum_{n>=2} c_n s^n (c_n = (2n-3)!!/(2^n n!)) to n = NT: to n = 9 its
// truncation error is below 3e-12 relative for s <= 0.05, and the launcher takes NT = 4
// where zl times the rest of the series is below 2^-28 revolution on the whole grid.
// The hardware sine and cosine take the reduced phase in revolutions.
template <int NT>
struct AsmHFastN {
    static_assert(NT == 4 || NT == 9, "series length");
    double lam_dfx, lam_dfy;  // lambda/(Mx dx), lambda/(My dy)
    double zl, half_zl;       // z/lambda, z/(2 lambda)
    float c0;                 // zl reduced to [-0.5, 0.5]
    int mx, my;
    struct Col {
        double a;
        float ca;  // c0 - reduced(zl*a/2)
    };
    __device__ __forceinline__ Col column(int p) const {
        const double x = (double)(p < mx / 2 ? p : p - mx) * lam_dfx;
        const double a = x * x;
        const double ta = half_zl * a;
        return Col{a, c0 - (float)(ta - rint(ta))};
    }
    struct Row {
        double b, hb;  // (lambda fy)^2 and zl*b/2
    };
    __device__ __forceinline__ Row row(int q) const {
        const double y = (double)(q < my / 2 ? q : q - my) * lam_dfy;
        const double b = y * y;
        return Row{b, half_zl * b};
    }
    __device__ __forceinline__ float2 operator()(const Col& c, const Row& rw) const {
        const double s = c.a + rw.b;
        double poly;
        if constexpr (NT == 9) {
            poly = 715.0 / 65536.0;
            poly = fma(poly, s, 429.0 / 32768.0);
            poly = fma(poly, s, 33.0 / 2048.0);
            poly = fma(poly, s, 21.0 / 1024.0);
            poly = fma(poly, s, 7.0 / 256.0);
            poly = fma(poly, s, 5.0 / 128.0);
        } else {
            poly = 5.0 / 128.0;
        }
        poly = fma(poly, s, 1.0 / 16.0);
        poly = fma(poly, s, 1.0 / 8.0);
        // zl*b/2 + zl*T(s), reduced (the exact fractional part), in FP64
        const double u = fma(zl * (s * s), poly, rw.hb);
        float r = c.ca - (float)__builtin_amdgcn_fract(u);
        r -= rintf(r);
        return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
    }
};
using AsmHFast = AsmHFastN<9>;

struct FresnelH {
    // the per-row factors are table reads: the column pass issues them before its forward
    // transform, so their latency hides behind it
    static constexpr bool kRowsEarly = true;
    const float2* __restrict__ hx;  // Mx entries, carries the constant C
    const float2* __restrict__ hy;  // My entries
    struct Col {
        float2 h;
    };
    struct Row {
        float2 h;
    };
    __device__ __forceinline__ Col column(int p) const { return Col{hx[p]}; }
    __device__ __forceinline__ Row row(int q) const { return Row{hy[q]}; }
    __device__ __forceinline__ float2 operator()(const Col& c, const Row& rw) const {
        return cmul(c.h, rw.h);
    }
};

// ---- per-plane transfer functions of a mixed batch -------------------------------------
//
// Planes of one geometry (sizes, pitch, flags) whose distance, wavelength or kind differ
// share the row passes; their column pass runs as one launch per transfer-function form
// present (fast ASM with the series to s^4, to s^9, Fresnel factors), each over its planes
// listed by buffer index, and each plane gets exactly the transfer function its single call
// would use. The kernel of each form is the single-plane kernel of that form.
template <class HF>
struct PlaneList {
    int n;
    int idx[kZChunk];  // buffer plane of launch plane k
    HF f[kZChunk];     // its transfer function
};

// Transfer function and buffer plane of launch plane pl: the functor itself and pl, or the
// list's entries.
template <class HF>
__device__ __forceinline__ const HF& plane_tf(const HF& hf, int) {
    return hf;
}
template <class HF>
__device__ __forceinline__ const HF& plane_tf(const PlaneList<HF>& t, int pl) {
    return t.f[pl];
}
template <class HF>
__device__ __forceinline__ int buffer_plane(const HF&, int pl) {
    return pl;
}
template <class HF>
__device__ __forceinline__ int buffer_plane(const PlaneList<HF>& t, int pl) {
    return t.idx[pl];
}

// Transfer functions whose per-row factors are memory reads say so with kRowsEarly.
template <class HF>
constexpr bool rows_early() {
    if constexpr (requires { HF::kRowsEarly; }) return HF::kRowsEarly;
    else return false;
}

// Column pass: forward FFT of COLS columns, multiplication by the transfer function,
// inverse FFT, in place; one (plane, column tile) item per block. LAY addresses the
// plane (row-major or tiled). With HALF the rows Ny..My-1 of the padded column are zero:
// they are neither loaded nor added in the first forward pass, and only rows < Ny of the
// result are computed to the end and stored. hscale (a power of two, 1 for complex64
// storage) multiplies the stored values; scaling by a power of two commutes exactly with
// the inverse transform, so this equals scaling the transfer function.
template <int M, bool HALF, class HF, class ST, class LAY>
__global__ __launch_bounds__(ColCfg<M>::THREADS) __attribute__((amdgpu_waves_per_eu(ColCfg<M>::WAVES_PER_EU))) void k_col(typename ST::E* __restrict__ buf,
                                                              int ny, int mx, int batch,
                                                              size_t plane, HF hf, float hscale,
                                                              const float2* __restrict__ tw,
                                                              LAY lay) {
    using C = ColCfg<M>;
    constexpr int E = C::E, T = C::T, P = C::P;
    using SE = typename ST::E;
    using PK = Pack<SE, P>;
    __shared__ float4 lds4[C::PAIRS * C::LDS_PAIR / 2];
    float2* lds = reinterpret_cast<float2*>(lds4);
    const int tid = threadIdx.x;
    const int pair = tid / T, j = tid % T;
    float2* my_lds = lds + pair * C::LDS_PAIR;
    TwCache<M, E> twc;
    twc.load(j, tw);
    const int ntiles = (mx + C::COLS - 1) / C::COLS;
    const int it = xcd_remap(blockIdx.x, gridDim.x);
    const int pl = it / ntiles, tile = it - pl * ntiles;
    const int col0 = (tile * C::PAIRS + pair) * P;  // first column of this thread (mx is even)
    // tiles of several pairs may overhang narrow planes (a one-pair tile never does)
    const bool active = C::PAIRS == 1 || col0 < mx;
    const int col = active ? col0 : 0;
    SE* base = buf + buffer_plane(hf, pl) * plane;
    const auto& hfp = plane_tf(hf, pl);  // this block's transfer function
    using PH = std::decay_t<decltype(hfp)>;
    float2 v[P][E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int y = j + r * T;
        const bool ld = active && (HALF ? (r < E / 2) : (y < ny));
        if (ld) {
            const PK t = *reinterpret_cast<const PK*>(base + lay.at(y, col));
#pragma unroll
            for (int p = 0; p < P; ++p) v[p][r] = ST::dec(t.e[p]);
        } else {
#pragma unroll
            for (int p = 0; p < P; ++p) v[p][r] = make_float2(0.f, 0.f);
        }
    }
    typename PH::Col hc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) hc[p] = hfp.column(col + p);
    // (at M = 8192 the extra registers cost more than the hidden latency: measured)
    constexpr bool EARLY = rows_early<PH>() && M <= 4096;
    typename PH::Row hre[EARLY ? E : 1];
    if constexpr (EARLY) {
#pragma unroll
        for (int r = 0; r < E; ++r) hre[r] = hfp.row(j + r * T);
    }
    if constexpr (HALF) fft_zpad<M, E, P, FWD, C::SPLIT>(v, my_lds, j, twc);
    else fft<M, E, P, FWD, C::SPLIT>(v, my_lds, j, twc);
#pragma unroll
    for (int r = 0; r < E; ++r) {
        typename PH::Row hr;
        if constexpr (EARLY) hr = hre[r];
        else hr = hfp.row(j + r * T);
#pragma unroll
        for (int p = 0; p < P; ++p) v[p][r] = cmul(v[p][r], hfp(hc[p], hr));
    }
    fft<M, E, P, INV, C::SPLIT>(v, my_lds, j, twc);
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int y = j + r * T;
        const bool st = active && (HALF ? (r < E / 2) : (y < ny));
        if (st) {
            PK t;
#pragma unroll
            for (int p = 0; p < P; ++p) t.e[p] = ST::enc(make_float2(v[p][r].x * hscale, v[p][r].y * hscale));
            *reinterpret_cast<PK*>(base + lay.at(y, col)) = t;
        }
    }
}

// Column pass for padded columns of length M = 2*MH with MH non-zero rows, as two
// transforms of length MH. With W = exp(-2 pi i/M), the padded forward transform's even
// bins are DFT_MH(x)[k] and its odd bins DFT_MH(x_n W^n)[k]; after multiplying by H(2k) and
// H(2k+1), the first MH outputs of the padded inverse transform are
// IDFT_MH(even)[n] + W^-n IDFT_MH(odd)[n]. One column per block of T = MH/16 threads, the
// two length-MH transforms sharing each thread's twiddles and 16-byte LDS slots (the pair
// of the two-column kernel), so a block needs half the threads and LDS of the length-M
// kernel and two blocks fit a CU. twm: the length-M table (the length-MH twiddles are its
// even entries).
template <int MH, class HF, class ST, class LAY>
__global__ __launch_bounds__(MH / 16) __attribute__((amdgpu_waves_per_eu(2))) void k_col_split(
    typename ST::E* __restrict__ buf, int ny, int mx, int batch, size_t plane, HF hf, float hscale,
    const float2* __restrict__ twm, LAY lay) {
    constexpr int E = 16, T = MH / E, P = 2;
    using SE = typename ST::E;
    __shared__ float4 lds4[lds_elems<MH>()];
    float2* lds = reinterpret_cast<float2*>(lds4);
    const int j = threadIdx.x;
    TwCache<MH, E> twc;
    twc.load(j, twm, 2);
    const int it = xcd_remap(blockIdx.x, gridDim.x);
    const int pl = it / mx, col = it - pl * mx;
    SE* base = buf + buffer_plane(hf, pl) * plane;
    const auto& hfp = plane_tf(hf, pl);
    using PH = std::decay_t<decltype(hfp)>;
    float2 v[P][E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int n = j + r * T;
        const float2 x = ST::dec(base[lay.at(n, col)]);
        v[0][r] = x;
        v[1][r] = cmul(x, twm[n]);
    }
    const typename PH::Col hc = hfp.column(col);
    fft<MH, E, P, FWD>(v, lds, j, twc);
    // opaque copies of j: the transfer function and the twiddles of the last step are
    // computed where they are used rather than held in registers through the transforms
    int jh = j;
    asm volatile("" : "+v"(jh));
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int k = jh + r * T;
#pragma unroll
        for (int p = 0; p < P; ++p) v[p][r] = cmul(v[p][r], hfp(hc, hfp.row(2 * k + p)));
    }
    fft<MH, E, P, INV>(v, lds, j, twc);
    int jj = j;
    asm volatile("" : "+v"(jj));
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int n = jj + r * T;
        const float2 o = cadd(v[0][r], ctw<INV>(v[1][r], twm[n]));
        base[lay.at(n, col)] = ST::enc(make_float2(o.x * hscale, o.y * hscale));
    }
}

}  // namespace cwo
