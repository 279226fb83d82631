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
    float2 v[1][E];
#pragma unroll
    for (int r = 0; r < E; ++r)
        v[0][r] = valid ? ST::dec(srow[j + r * T]) : make_float2(0.f, 0.f);
    fft<M, E, 1, INV>(v, my_lds, j, tw);
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
    if (num) {
        // deterministic per-row sum: lane partials through LDS, summed in index order
        double* red = reinterpret_cast<double*>(my_lds);
        lds_barrier();
        red[j] = acc;
        lds_barrier();
        if (j == 0 && valid) {
            double t = 0.0;
            for (int i = 0; i < T; ++i) t += red[i];
            num[row] = t;
        }
        lds_barrier();
    }
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
    fft<M, E, 1, FWD>(v, my_lds, j, tw);
    if (valid) {
#pragma unroll
        for (int r = 0; r < E; ++r) srow[j + r * T] = ST::enc(v[0][r]);
    }
}

// den = sum(amp^2) in FP64 by one block (deterministic order), then one block per
// iteration sums its row partials.
__global__ __launch_bounds__(256) void k_gs_den(const float* __restrict__ amp, double* den,
                                                long long count) {
    __shared__ double red[256];
    double t = 0.0;
    for (long long i = threadIdx.x; i < count; i += 256) {
        const double a = amp[i];
        t += a * a;
    }
    red[threadIdx.x] = t;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *den = red[0];
}

__global__ __launch_bounds__(256) void k_gs_errors(const double* __restrict__ num,
                                                   const double* __restrict__ den,
                                                   float* __restrict__ errors, int ny) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    double t = 0.0;
    for (int i = threadIdx.x; i < ny; i += 256) t += num[(size_t)k * ny + i];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) errors[k] = (float)sqrt(red[0] / *den);
}

// ---- host launchers ------------------------------------------------------------

namespace {
template <class ST>
hipError_t row_gs_t(void* spec, const float* amp, float2* out, double* num, int nx, int ny,
                    int mx, float scale, const float* dyn_inv, float fwd_scale,
                    const float* dyn_fwd, const float2* tw, hipStream_t s) {
    using SE = typename ST::E;
    const bool half = (mx == 2 * nx);
    CWO_DISPATCH_M(mx, {
        using C = RowCfg<MM>;
        dim3 grid((ny + C::RPB - 1) / C::RPB);
        if (half)
            hipLaunchKernelGGL((k_row_gs<MM, true, ST>), grid, dim3(C::THREADS), 0, s, (SE*)spec,
                               amp, out, num, nx, ny, scale, dyn_inv, fwd_scale, dyn_fwd, tw);
        else
            hipLaunchKernelGGL((k_row_gs<MM, false, ST>), grid, dim3(C::THREADS), 0, s, (SE*)spec,
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
                                   gsc.fwd_scale, gsc.dyn_fwd, tw, s);
        case 1:
            return row_gs_t<StF16>(spec, amp, out, num, nx, ny, mx, gsc.scale, gsc.dyn_inv,
                                   gsc.fwd_scale, gsc.dyn_fwd, tw, s);
        case 2:
            return row_gs_t<StBF16>(spec, amp, out, num, nx, ny, mx, gsc.scale, gsc.dyn_inv,
                                    gsc.fwd_scale, gsc.dyn_fwd, tw, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_gs_errors(const double* num, const float* amp, double* den_work, float* errors,
                            int nx, int ny, int iters, hipStream_t s) {
    hipLaunchKernelGGL(k_gs_den, dim3(1), dim3(256), 0, s, amp, den_work, (long long)nx * ny);
    hipLaunchKernelGGL(k_gs_errors, dim3(iters), dim3(256), 0, s, num, (const double*)den_work,
                       errors, ny);
    return hipGetLastError();
}

}  // namespace cwo
