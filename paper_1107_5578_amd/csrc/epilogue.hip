// Field epilogues of the paper's examples: intensity |u|^2 and its min-max scale to
// 0..top (Sec. 3.1, Eq. norm; the 256-step image for top = 255), the phase of a field
// (the kinoform, Sec. 7.1) and a phase field back to a complex one. Streaming kernels,
// grid-stride over n elements.
//
// The FP32 operation order is fixed (products and sums rounded separately: contraction
// into fused multiply-adds is switched off where it matters; the scale in the order Eq.
// norm prints it, (I - min), then / (max - min) (IEEE division), then * top), so the
// 8-bit codes, which floating point decides, are reproducible.

#include "kernel_common.hpp"

namespace cwo {

constexpr int kEpiThreads = 256;

__global__ __launch_bounds__(kEpiThreads) void k_intensity(const float2* __restrict__ in,
                                                           float* __restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kEpiThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kEpiThreads) {
#pragma clang fp contract(off)
        const float2 v = in[i];
        out[i] = v.x * v.x + v.y * v.y;
    }
}

__global__ __launch_bounds__(kEpiThreads) void k_phase(const float2* __restrict__ in,
                                                       float* __restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kEpiThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kEpiThreads) {
        const float2 v = in[i];
        out[i] = atan2f(v.y, v.x);
    }
}

__global__ __launch_bounds__(kEpiThreads) void k_polar(const float* __restrict__ phi,
                                                       const float* __restrict__ amp,
                                                       float2* __restrict__ out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kEpiThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kEpiThreads) {
        float s, c;
        sincosf(phi[i], &s, &c);
        const float a = amp ? amp[i] : 1.0f;
        out[i] = make_float2(a * c, a * s);
    }
}

// per-block minimum and maximum (part[2b], part[2b + 1])
__global__ __launch_bounds__(kEpiThreads) void k_minmax_partial(const float* __restrict__ in,
                                                                size_t n,
                                                                float* __restrict__ part) {
    __shared__ float lo[kEpiThreads], hi[kEpiThreads];
    float a = INFINITY, b = -INFINITY;
    for (size_t i = (size_t)blockIdx.x * kEpiThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kEpiThreads) {
        const float v = in[i];
        a = fminf(a, v);
        b = fmaxf(b, v);
    }
    lo[threadIdx.x] = a;
    hi[threadIdx.x] = b;
    __syncthreads();
    for (int s = kEpiThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            lo[threadIdx.x] = fminf(lo[threadIdx.x], lo[threadIdx.x + s]);
            hi[threadIdx.x] = fmaxf(hi[threadIdx.x], hi[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = lo[0];
        part[2 * blockIdx.x + 1] = hi[0];
    }
}

// mm[0] = min, mm[1] = max over the partials; mm[2] = max - min; mm[3] = top
__global__ __launch_bounds__(kEpiThreads) void k_minmax_final(const float* __restrict__ part,
                                                              int np, float top,
                                                              float* __restrict__ mm) {
    __shared__ float lo[kEpiThreads], hi[kEpiThreads];
    float a = INFINITY, b = -INFINITY;
    for (int i = threadIdx.x; i < np; i += kEpiThreads) {
        a = fminf(a, part[2 * i]);
        b = fmaxf(b, part[2 * i + 1]);
    }
    lo[threadIdx.x] = a;
    hi[threadIdx.x] = b;
    __syncthreads();
    for (int s = kEpiThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            lo[threadIdx.x] = fminf(lo[threadIdx.x], lo[threadIdx.x + s]);
            hi[threadIdx.x] = fmaxf(hi[threadIdx.x], hi[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma clang fp contract(off)
        mm[0] = lo[0];
        mm[1] = hi[0];
        mm[2] = hi[0] - lo[0];
        mm[3] = top;
    }
}

template <bool U8>
__global__ __launch_bounds__(kEpiThreads) void k_scale(const float* __restrict__ in, size_t n,
                                                       const float* __restrict__ mm,
                                                       void* __restrict__ out) {
    const float mn = mm[0], range = mm[2], top = mm[3];
    for (size_t i = (size_t)blockIdx.x * kEpiThreads + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kEpiThreads) {
#pragma clang fp contract(off)
        // a constant field (max == min) scales to 0
        const float v = range == 0.0f ? 0.0f : ((in[i] - mn) / range) * top;
        if constexpr (U8) {
            const float q = fminf(fmaxf(rintf(v), 0.0f), 255.0f);
            static_cast<uint8_t*>(out)[i] = (uint8_t)q;
        } else {
            static_cast<float*>(out)[i] = v;
        }
    }
}

static unsigned epi_grid(size_t n) {
    const size_t b = (n + kEpiThreads - 1) / kEpiThreads;
    return (unsigned)(b < (size_t)kRangeBlocks * 4 ? (b ? b : 1) : (size_t)kRangeBlocks * 4);
}

hipError_t launch_intensity(const float2* in, float* out, size_t n, hipStream_t s) {
    launch_kernel(k_intensity, dim3(epi_grid(n)), dim3(kEpiThreads), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_phase(const float2* in, float* out, size_t n, hipStream_t s) {
    launch_kernel(k_phase, dim3(epi_grid(n)), dim3(kEpiThreads), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_polar(const float* phi, const float* amp, float2* out, size_t n, hipStream_t s) {
    launch_kernel(k_polar, dim3(epi_grid(n)), dim3(kEpiThreads), 0, s, phi, amp, out, n);
    return hipGetLastError();
}

hipError_t launch_scale(const float* in, size_t n, float top, bool u8, void* out, float* work,
                        hipStream_t s) {
    const unsigned nb = epi_grid(n) < (unsigned)kRangeBlocks ? epi_grid(n) : (unsigned)kRangeBlocks;
    float* part = work + 4;
    launch_kernel(k_minmax_partial, dim3(nb), dim3(kEpiThreads), 0, s, in, n, part);
    launch_kernel(k_minmax_final, dim3(1), dim3(kEpiThreads), 0, s, part, (int)nb, top, work);
    if (u8)
        launch_kernel(k_scale<true>, dim3(epi_grid(n)), dim3(kEpiThreads), 0, s, in, n,
                           (const float*)work, out);
    else
        launch_kernel(k_scale<false>, dim3(epi_grid(n)), dim3(kEpiThreads), 0, s, in, n,
                           (const float*)work, out);
    return hipGetLastError();
}

}  // namespace cwo
