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
//             in FP64 by direct summation.
#include <cstddef>
#include <cstdint>
#include <utility>

#include "fft_device.hpp"
#include "launch.hpp"

namespace cwo {

// ---- configuration per transform length --------------------------------------

template <int M>
struct RowCfg {
    static constexpr int E = (M == 512 || M == 8192) ? 32 : 16;
    static constexpr int T = M / E;
    static constexpr int RPB = (T >= 256) ? 1 : 256 / T;  // rows per block
    static constexpr int THREADS = T * RPB;
};

template <int M>
struct ColCfg {
    static constexpr int E = (M == 512 || M == 8192) ? 32 : 16;
    static constexpr int T = M / E;
    // columns per block: keep the LDS exchange buffer near 72 KiB and at most 512 threads
    static constexpr int BY_LDS = (72 * 1024) / (lds_elems<M>() * 8);
    static constexpr int BY_THR = 512 / T;
    static constexpr int C0 = BY_LDS < BY_THR ? BY_LDS : BY_THR;
    static constexpr int C = C0 < 1 ? 1 : (C0 > 16 ? 16 : C0);
    static constexpr int THREADS = T * C;
};

// Consecutive workgroup ids are dispatched round-robin over the 8 XCDs, which
// have separate L2 caches. Remap so that each XCD works on a contiguous range
// of tiles; neighbouring tiles share cache lines.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
    if ((nblocks & 7) != 0) return bid;
    const int per = nblocks >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// ---- row forward: zero-pad + FFT --------------------------------------------

template <int M, bool HALF>
__global__ __launch_bounds__(RowCfg<M>::THREADS) void k_row_fwd(const float2* __restrict__ in,
                                                                  float2* __restrict__ out, int nx,
                                                                  int ny, size_t in_plane,
                                                                  size_t out_plane,
                                                                  const float2* __restrict__ tw) {
    using C = RowCfg<M>;
    constexpr int E = C::E, T = C::T;
    __shared__ float2 lds[C::RPB * lds_elems<M>()];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    const int row = blockIdx.x * C::RPB + sub;
    const bool valid = row < ny;
    const float2* src = in + blockIdx.y * in_plane + (size_t)row * nx;
    float2 v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = j + r * T;
        if constexpr (HALF) {
            // M == 2*nx: exactly the first E/2 registers hold field values
            v[r] = (r < E / 2 && valid) ? src[x] : make_float2(0.f, 0.f);
        } else {
            v[r] = (valid && x < nx) ? src[x] : make_float2(0.f, 0.f);
        }
    }
    fft<M, E, FWD>(v, lds + sub * lds_elems<M>(), j, tw);
    if (valid) {
        float2* dst = out + blockIdx.y * out_plane + (size_t)row * M;
#pragma unroll
        for (int r = 0; r < E; ++r) dst[j + r * T] = v[r];
    }
}

// ---- column pass: FFT, transfer function, IFFT, crop --------------------------

struct AsmH {
    double dfx, dfy;  // frequency pitches 1/(Mx dx), 1/(My dy)
    double lam;       // wavelength
    double zl;        // z / lambda: phase in revolutions per unit sqrt(1 - s)
    int mx, my;
    __device__ __forceinline__ float2 operator()(int p, int q) const {
        const double pp = (double)(p < mx / 2 ? p : p - mx);
        const double qq = (double)(q < my / 2 ? q : q - my);
        // s = (lambda*fx)^2 + (lambda*fy)^2 with fx = p'*dfx, evaluated without contraction
        const double ax = __dmul_rn(lam, __dmul_rn(pp, dfx));
        const double ay = __dmul_rn(lam, __dmul_rn(qq, dfy));
        const double s = __dadd_rn(__dmul_rn(ay, ay), __dmul_rn(ax, ax));
        if (!(s <= 1.0)) return make_float2(0.f, 0.f);  // evanescent bin
        const double t = zl * __dsqrt_rn(1.0 - s);       // revolutions
        const float r = (float)(t - rint(t));            // [-0.5, 0.5]
        float sn, cs;
        sincospif(2.0f * r, &sn, &cs);
        return make_float2(cs, sn);
    }
};

struct FresnelH {
    const float2* __restrict__ hx;  // Mx entries, carries the constant C
    const float2* __restrict__ hy;  // My entries
    __device__ __forceinline__ float2 operator()(int p, int q) const { return cmul(hx[p], hy[q]); }
};

template <int M, bool HALF, class HF>
__global__ __launch_bounds__(ColCfg<M>::THREADS) void k_col(float2* __restrict__ buf, int ny,
                                                              int mx, size_t plane, HF hf,
                                                              const float2* __restrict__ tw) {
    using C = ColCfg<M>;
    constexpr int E = C::E, T = C::T;
    __shared__ float2 lds[C::C * lds_elems<M>()];
    const int tid = threadIdx.x;
    const int c = tid % C::C, j = tid / C::C;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int col = blk * C::C + c;  // mx is a multiple of C (both powers of two, C <= mx)
    float2* base = buf + blockIdx.y * plane + col;
    float2 v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int y = j + r * T;
        if constexpr (HALF) v[r] = (r < E / 2) ? base[(size_t)y * mx] : make_float2(0.f, 0.f);
        else v[r] = (y < ny) ? base[(size_t)y * mx] : make_float2(0.f, 0.f);
    }
    float2* my_lds = lds + c * lds_elems<M>();
    fft<M, E, FWD>(v, my_lds, j, tw);
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = cmul(v[r], hf(col, j + r * T));
    fft<M, E, INV>(v, my_lds, j, tw);
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int y = j + r * T;
        if constexpr (HALF) {
            if (r < E / 2) base[(size_t)y * mx] = v[r];
        } else {
            if (y < ny) base[(size_t)y * mx] = v[r];
        }
    }
}

// ---- row inverse: IFFT + crop + normalisation ---------------------------------

template <int M, bool HALF>
__global__ __launch_bounds__(RowCfg<M>::THREADS) void k_row_inv(const float2* __restrict__ in,
                                                                  float2* __restrict__ out, int nx,
                                                                  int ny, size_t in_plane,
                                                                  size_t out_plane, float scale,
                                                                  const float2* __restrict__ tw) {
    using C = RowCfg<M>;
    constexpr int E = C::E, T = C::T;
    __shared__ float2 lds[C::RPB * lds_elems<M>()];
    const int tid = threadIdx.x;
    const int sub = tid / T, j = tid % T;
    const int row = blockIdx.x * C::RPB + sub;
    const bool valid = row < ny;
    const float2* src = in + blockIdx.y * in_plane + (size_t)(valid ? row : 0) * M;
    float2 v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = valid ? src[j + r * T] : make_float2(0.f, 0.f);
    fft<M, E, INV>(v, lds + sub * lds_elems<M>(), j, tw);
    if (valid) {
        float2* dst = out + blockIdx.y * out_plane + (size_t)row * nx;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int x = j + r * T;
            const float2 o = make_float2(v[r].x * scale, v[r].y * scale);
            if constexpr (HALF) {
                if (r < E / 2) dst[x] = o;
            } else {
                if (x < nx) dst[x] = o;
            }
        }
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

// Sampled 1-D chirp of the Fresnel impulse response on the padded axis:
// h[d] = exp(i * a * (s(d)*pitch)^2), s(d) = d for d < n, d - m otherwise,
// a = pi/(lambda z); the phase is evaluated in revolutions (a/pi)(...)/2 and reduced.
__global__ void k_chirp(double2* h, int m, int n, double pitch, double half_rev_per_m2) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= m) return;
    const double off = (double)(d < n ? d : d - m) * pitch;
    const double t = half_rev_per_m2 * (off * off);  // revolutions = (1/(2 lambda z)) x^2
    const double r = t - rint(t);
    double s, c;
    sincospi(2.0 * r, &s, &c);
    h[d] = make_double2(c, s);
}

// tw64[k] = exp(-2*pi*i*k/M) in FP64 (for the FP64 chirp transforms)
__global__ void k_twiddles64(double2* tw, int m) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    double s, c;
    sincospi(2.0 * (double)k / (double)m, &s, &c);
    tw[k] = make_double2(c, -s);
}

// Hx[p] = coef * sum_d h[d] * exp(-2*pi*i*((p*d) mod m)/m), FP64 accumulation.
// One block of 256 threads per output bin.
__global__ __launch_bounds__(256) void k_chirp_dft(const double2* __restrict__ h,
                                                   const double2* __restrict__ tw64,
                                                   float2* __restrict__ out, int m, double coef_re,
                                                   double coef_im) {
    __shared__ double red[2][256];
    const int p = blockIdx.x;
    double ar = 0.0, ai = 0.0;
    for (int d = threadIdx.x; d < m; d += 256) {
        const int idx = (int)(((long long)p * d) & (m - 1));
        const double2 w = tw64[idx];
        const double2 x = h[d];
        ar += x.x * w.x - x.y * w.y;
        ai += x.x * w.y + x.y * w.x;
    }
    red[0][threadIdx.x] = ar;
    red[1][threadIdx.x] = ai;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double sr = red[0][0], si = red[1][0];
        out[p] = make_float2((float)(sr * coef_re - si * coef_im), (float)(sr * coef_im + si * coef_re));
    }
}

// ---- host launchers ------------------------------------------------------------

#define CWO_DISPATCH_M(M_, BODY)              \
    switch (M_) {                             \
        case 16: { constexpr int MM = 16; BODY; } break;     \
        case 32: { constexpr int MM = 32; BODY; } break;     \
        case 64: { constexpr int MM = 64; BODY; } break;     \
        case 128: { constexpr int MM = 128; BODY; } break;   \
        case 256: { constexpr int MM = 256; BODY; } break;   \
        case 512: { constexpr int MM = 512; BODY; } break;   \
        case 1024: { constexpr int MM = 1024; BODY; } break; \
        case 2048: { constexpr int MM = 2048; BODY; } break; \
        case 4096: { constexpr int MM = 4096; BODY; } break; \
        case 8192: { constexpr int MM = 8192; BODY; } break; \
        default: return hipErrorInvalidValue;                 \
    }

hipError_t launch_twiddles(float2* tw, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_twiddles, dim3((m + 255) / 256), dim3(256), 0, s, tw, m);
    return hipGetLastError();
}

hipError_t launch_row_fwd(const float2* in, float2* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, const float2* tw, hipStream_t s) {
    const bool half = (mx == 2 * nx);
    CWO_DISPATCH_M(mx, {
        using C = RowCfg<MM>;
        dim3 grid((ny + C::RPB - 1) / C::RPB, batch);
        if (half)
            hipLaunchKernelGGL((k_row_fwd<MM, true>), grid, dim3(C::THREADS), 0, s, in, out, nx, ny,
                               in_plane, out_plane, tw);
        else
            hipLaunchKernelGGL((k_row_fwd<MM, false>), grid, dim3(C::THREADS), 0, s, in, out, nx,
                               ny, in_plane, out_plane, tw);
    });
    return hipGetLastError();
}

template <class HF>
static hipError_t launch_col_impl(float2* buf, int ny, int my, int mx, int batch, size_t plane,
                                  const HF& hf, const float2* tw, hipStream_t s) {
    const bool half = (my == 2 * ny);
    CWO_DISPATCH_M(my, {
        using C = ColCfg<MM>;
        if (mx % C::C != 0) return hipErrorInvalidValue;
        dim3 grid(mx / C::C, batch);
        if (half)
            hipLaunchKernelGGL((k_col<MM, true, HF>), grid, dim3(C::THREADS), 0, s, buf, ny, mx,
                               plane, hf, tw);
        else
            hipLaunchKernelGGL((k_col<MM, false, HF>), grid, dim3(C::THREADS), 0, s, buf, ny, mx,
                               plane, hf, tw);
    });
    return hipGetLastError();
}

hipError_t launch_col_asm(float2* buf, int ny, int my, int mx, int batch, size_t plane,
                          const AsmScalars& a, const float2* tw, hipStream_t s) {
    AsmH hf{a.dfx, a.dfy, a.lam, a.zl, mx, my};
    return launch_col_impl(buf, ny, my, mx, batch, plane, hf, tw, s);
}

hipError_t launch_col_fresnel(float2* buf, int ny, int my, int mx, int batch, size_t plane,
                              const float2* hx, const float2* hy, const float2* tw, hipStream_t s) {
    FresnelH hf{hx, hy};
    return launch_col_impl(buf, ny, my, mx, batch, plane, hf, tw, s);
}

hipError_t launch_row_inv(const float2* in, float2* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, float scale, const float2* tw,
                          hipStream_t s) {
    const bool half = (mx == 2 * nx);
    CWO_DISPATCH_M(mx, {
        using C = RowCfg<MM>;
        dim3 grid((ny + C::RPB - 1) / C::RPB, batch);
        if (half)
            hipLaunchKernelGGL((k_row_inv<MM, true>), grid, dim3(C::THREADS), 0, s, in, out, nx, ny,
                               in_plane, out_plane, scale, tw);
        else
            hipLaunchKernelGGL((k_row_inv<MM, false>), grid, dim3(C::THREADS), 0, s, in, out, nx,
                               ny, in_plane, out_plane, scale, tw);
    });
    return hipGetLastError();
}

hipError_t launch_fresnel_axis(double2* work, float2* out, int m, int n, double pitch,
                               double lam_z, double coef_re, double coef_im, hipStream_t s) {
    // work holds 2*m FP64 complex values: the chirp, then the FP64 twiddle table
    const double half_rev_per_m2 = 0.5 / lam_z;  // pi/(lambda z) rad = 1/(2 lambda z) rev
    double2* chirp = work;
    double2* tw64 = work + m;
    hipLaunchKernelGGL(k_twiddles64, dim3((m + 255) / 256), dim3(256), 0, s, tw64, m);
    hipLaunchKernelGGL(k_chirp, dim3((m + 255) / 256), dim3(256), 0, s, chirp, m, n, pitch,
                       half_rev_per_m2);
    hipLaunchKernelGGL(k_chirp_dft, dim3(m), dim3(256), 0, s, (const double2*)chirp,
                       (const double2*)tw64, out, m, coef_re, coef_im);
    return hipGetLastError();
}

}  // namespace cwo
