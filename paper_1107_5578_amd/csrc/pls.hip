// HIP kernels of the point-light-source (PLS) field and hologram: direct sums of
// Fresnel wavelets over N object points (Sec. 2.4, Eqs. pls_fre and pls_fre_cgh).
//
// Every (pixel, point) term evaluates its phase r^2/(2 lambda z_j) in revolutions in
// FP64, takes its fractional part in FP64 (one exact instruction) and the hardware
// cosine (and sine) of that remainder rounded to FP32, which work in revolutions. The sum
// is arithmetic-bound (no transform, O(N Nx Ny) terms): points are staged through LDS in
// chunks read by all threads at once (one broadcast address per wavefront), each thread
// owns kPlsPx pixels of a row, and the row's y distance to the point is shared by them.
// Partial sums over a chunk are FP32, the running sum across chunks FP64.

#include "kernel_common.hpp"

namespace cwo {

namespace {

constexpr int kPlsThreads = 256;
constexpr int kPlsPx = 4;                       // pixels per thread, kPlsThreads apart
constexpr int kPlsTile = kPlsThreads * kPlsPx;  // pixels of one row per block
constexpr int kPlsChunk = 512;                  // points per LDS stage (16 KB)

// One object point in absolute coordinates: x_j, y_j [m], c_j = 1/(2 lambda z_j)
// [revolutions per m^2] and its amplitude A_j (32 bytes).
struct PlsPoint {
    double x, y, c;
    float a, pad;
};

__global__ __launch_bounds__(256) void k_pls_points(const float4* __restrict__ in, int n,
                                                    PlsPoint* __restrict__ out, double ox,
                                                    double oy, double oz, double lam) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 p = in[i];
    out[i] = PlsPoint{ox + (double)p.x, oy + (double)p.y, 0.5 / (lam * (oz + (double)p.z)), p.w,
                      0.f};
}

// FIELD false: out is float [ny][nx], I = sum_j A_j cos(2 pi r_j).
// FIELD true: out is complex64 [ny][nx], u = C sum_j A_j exp(2 pi i r_j), C = (cre, cim).
template <bool FIELD>
__global__ __launch_bounds__(kPlsThreads) void k_pls(const PlsPoint* __restrict__ pts, int npts,
                                                     void* __restrict__ out, int nx, int ny,
                                                     double px, double py, double cre,
                                                     double cim) {
    __shared__ PlsPoint sp[kPlsChunk];
    const int row = blockIdx.y;
    const int x0 = blockIdx.x * kPlsTile + threadIdx.x;
    const double y = (double)(row - ny / 2) * py;
    double xs[kPlsPx];
#pragma unroll
    for (int k = 0; k < kPlsPx; ++k) xs[k] = (double)(x0 + k * kPlsThreads - nx / 2) * px;
    double sre[kPlsPx], sim[kPlsPx];
#pragma unroll
    for (int k = 0; k < kPlsPx; ++k) sre[k] = sim[k] = 0.0;
    for (int base = 0; base < npts; base += kPlsChunk) {
        const int cnt = npts - base < kPlsChunk ? npts - base : kPlsChunk;
        __syncthreads();
        for (int i = threadIdx.x; i < cnt; i += kPlsThreads) sp[i] = pts[base + i];
        __syncthreads();
        float cre_f[kPlsPx], cim_f[kPlsPx];
#pragma unroll
        for (int k = 0; k < kPlsPx; ++k) cre_f[k] = cim_f[k] = 0.f;
        for (int j = 0; j < cnt; ++j) {
            const PlsPoint q = sp[j];
            const double dy = y - q.y;
            const double dy2 = dy * dy;
            const float a = q.a;
#pragma unroll
            for (int k = 0; k < kPlsPx; ++k) {
                const double dx = xs[k] - q.x;
                const double t = q.c * fma(dx, dx, dy2);
                const float r = (float)__builtin_amdgcn_fract(t);  // [0, 1) revolutions
                cre_f[k] = fmaf(a, __builtin_amdgcn_cosf(r), cre_f[k]);
                if constexpr (FIELD) cim_f[k] = fmaf(a, __builtin_amdgcn_sinf(r), cim_f[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < kPlsPx; ++k) {
            sre[k] += (double)cre_f[k];
            if constexpr (FIELD) sim[k] += (double)cim_f[k];
        }
    }
#pragma unroll
    for (int k = 0; k < kPlsPx; ++k) {
        const int x = x0 + k * kPlsThreads;
        if (x >= nx) continue;
        const size_t o = (size_t)row * nx + x;
        if constexpr (FIELD) {
            static_cast<float2*>(out)[o] =
                make_float2((float)(cre * sre[k] - cim * sim[k]), (float)(cre * sim[k] + cim * sre[k]));
        } else {
            static_cast<float*>(out)[o] = (float)sre[k];
        }
    }
}

}  // namespace

hipError_t launch_pls(const float* points, int npts, void* work, void* out, bool field,
                      const PlsParams& pp, hipStream_t s) {
    PlsPoint* recs = static_cast<PlsPoint*>(work);
    if (npts > 0)
        launch_kernel(k_pls_points, dim3((npts + 255) / 256), dim3(256), 0, s,
                           reinterpret_cast<const float4*>(points), npts, recs, pp.ox, pp.oy,
                           pp.oz, pp.lam);
    const dim3 grid((pp.nx + kPlsTile - 1) / kPlsTile, pp.ny);
    if (field)
        launch_kernel(k_pls<true>, grid, dim3(kPlsThreads), 0, s, (const PlsPoint*)recs, npts,
                           out, pp.nx, pp.ny, pp.px, pp.py, pp.cre, pp.cim);
    else
        launch_kernel(k_pls<false>, grid, dim3(kPlsThreads), 0, s, (const PlsPoint*)recs, npts,
                           out, pp.nx, pp.ny, pp.px, pp.py, pp.cre, pp.cim);
    return hipGetLastError();
}

size_t pls_work_bytes(int npts) { return (size_t)(npts > 0 ? npts : 1) * sizeof(PlsPoint); }

}  // namespace cwo
