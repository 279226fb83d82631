// HIP kernels of the Fresnel transfer-function factor tables.

#include "kernel_common.hpp"

namespace cwo {

// ---- Fresnel transfer-function factors ---------------------------------------
//
// The FFT of the sampled impulse response h_F(m, n) = hx(m) hy(n) is the outer
// product of two 1-D transforms, each computed here by an FP64 FFT with an FP64
// twiddle table (every twiddle correct to an ulp).

// tw64[i] = exp(-2*pi*i*d/m) for the x axis (i < mx) then the y axis
__global__ void k_twiddles64(double2* tw, int mx, int my) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= mx + my) return;
    const bool xa = i < mx;
    const int d = xa ? i : i - mx, m = xa ? mx : my;
    double sn, cs;
    sincospi(2.0 * (double)d / (double)m, &sn, &cs);
    tw[i] = make_double2(cs, -sn);
}

// One 1-D Fresnel factor per block (blockIdx.x = axis, blockIdx.y = plane): the sampled
// chirp h(d) = exp(i*pi*(s(d)*pitch)^2/(lambda z)) with signed offsets s(d), its length-m
// DFT in FP64 (radix-2, decimation in time from bit-reversed order, in LDS), times the
// plane constant C_k on the x axis, rounded to complex64. The chirp phase is reduced
// modulo one revolution in FP64 before the sine and cosine.
constexpr int kChirpMaxM = 8192;
__global__ __launch_bounds__(256) void k_chirp_fft(const double2* __restrict__ tw64,
                                                   float2* __restrict__ out, FresnelPlanes fp) {
    __shared__ double2 a[kChirpMaxM];
    const bool xa = blockIdx.x == 0;
    const int k = blockIdx.y;
    const int m = xa ? fp.mx : fp.my, n = xa ? fp.nx : fp.ny;
    const double pitch = xa ? fp.dx : fp.dy;
    const double2* w = tw64 + (xa ? 0 : fp.mx);
    const int lg = 31 - __clz(m);
    for (int d = threadIdx.x; d < m; d += blockDim.x) {
        const double off = (double)(d < n ? d : d - m) * pitch;
        const double t = fp.inv2lz[k] * (off * off);
        const double r = t - rint(t);
        double sn, cs;
        sincospi(2.0 * r, &sn, &cs);
        a[__brev((unsigned)d) >> (32 - lg)] = make_double2(cs, sn);
    }
    __syncthreads();
    for (int half = 1; half < m; half <<= 1) {
        const int step = m / (2 * half);  // W_{2 half}^pos = W_m^(pos*step)
        for (int t = threadIdx.x; t < m / 2; t += blockDim.x) {
            const int pos = t & (half - 1);
            const int i = 2 * (t - pos) + pos;
            const double2 wv = w[pos * step];
            const double2 x = a[i], y = a[i + half];
            const double yr = y.x * wv.x - y.y * wv.y, yi = y.x * wv.y + y.y * wv.x;
            a[i] = make_double2(x.x + yr, x.y + yi);
            a[i + half] = make_double2(x.x - yr, x.y - yi);
        }
        __syncthreads();
    }
    const double cr = xa ? fp.cre[k] : 1.0, ci = xa ? fp.cim[k] : 0.0;
    float2* o = out + (size_t)k * (fp.mx + fp.my) + (xa ? 0 : fp.mx);
    for (int p = threadIdx.x; p < m; p += blockDim.x) {
        const double2 v = a[p];
        o[p] = make_float2((float)(v.x * cr - v.y * ci), (float)(v.x * ci + v.y * cr));
    }
}

// Analytic factors: one thread per entry (blockIdx.y = plane). Entry i < mx is Hx at
// fx = s(i)/(mx dx), the rest Hy at fy = s(i - mx)/(my dy), with s(p) = p for p < m/2 and
// p - m above; the phase -lambda z f^2 / 2 (revolutions) is reduced modulo one in FP64
// before the sine and cosine, then Hx takes the plane constant.
__global__ __launch_bounds__(256) void k_fresnel_tf(float2* __restrict__ out, FresnelPlanes fp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= fp.mx + fp.my) return;
    const bool xa = i < fp.mx;
    const int d = xa ? i : i - fp.mx, m = xa ? fp.mx : fp.my;
    const double f = (double)(d < m / 2 ? d : d - m) / ((double)m * (xa ? fp.dx : fp.dy));
    const double t = -fp.hlz[k] * (f * f);
    const double r = t - rint(t);
    double sn, cs;
    sincospi(2.0 * r, &sn, &cs);
    const double cr = xa ? fp.cre[k] : 1.0, ci = xa ? fp.cim[k] : 0.0;
    out[(size_t)k * (fp.mx + fp.my) + i] =
        make_float2((float)(cs * cr - sn * ci), (float)(cs * ci + sn * cr));
}

// ---- host launchers ------------------------------------------------------------

hipError_t launch_fresnel_planes(double2* work, float2* out, const FresnelPlanes& fp,
                                 hipStream_t s) {
    if (fp.mx > kChirpMaxM || fp.my > kChirpMaxM) return hipErrorInvalidValue;
    if (fp.analytic) {
        launch_kernel(k_fresnel_tf, dim3((fp.mx + fp.my + 255) / 256, fp.nz), dim3(256), 0, s,
                           out, fp);
        return hipGetLastError();
    }
    const int len = fp.mx + fp.my;
    double2* tw64 = work;
    launch_kernel(k_twiddles64, dim3((len + 255) / 256), dim3(256), 0, s, tw64, fp.mx, fp.my);
    launch_kernel(k_chirp_fft, dim3(2, fp.nz), dim3(256), 0, s, (const double2*)tw64, out, fp);
    return hipGetLastError();
}

}  // namespace cwo
