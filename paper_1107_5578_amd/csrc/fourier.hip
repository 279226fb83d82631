// Fresnel diffraction in Fourier form (Sec. 2.1.2, Eqs. fre_fourier1 - fre_fourier3): one
// unpadded 2-D FFT of the field times a chirp, then the destination chirp and the
// constant dx dy exp(i k z)/(i lambda z).
//
// Sample positions are centred (index j is coordinate (j - N/2) * pitch) and the
// destination pitch is lambda z/(N dx1). With N/2 even the centred DFT is the plain DFT
// between two (-1)^j sign patterns, which are folded into the chirp factors, so the
// path is two kernels working in place on the output plane:
//   ff_row : per row, load N values times prex[x] * prey[y], forward FFT, store;
//   ff_col : per column, forward FFT, times postx[x] * posty[y], store.
// The four 1-D factor tables are computed in FP64 (phases reduced modulo one revolution)
// and rounded once to complex64.

#include "kernel_common.hpp"

namespace cwo {

// tabs = [prex (nx) | prey (ny) | postx (nx) | posty (ny)]
__global__ void k_ff_tables(float2* __restrict__ tabs, FourierPlan fp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int len = fp.nx + fp.ny;
    if (i >= 2 * len) return;
    const bool post = i >= len;
    const int k = post ? i - len : i;
    const bool xa = k < fp.nx;
    const int j = xa ? k : k - fp.nx;
    const int n = xa ? fp.nx : fp.ny;
    const double pitch = post ? (xa ? fp.dx2 : fp.dy2) : (xa ? fp.dx : fp.dy);
    const double x = (double)(j - n / 2) * pitch;
    const double t = (x * x) * fp.inv2lz;  // revolutions of exp(i pi x^2/(lambda z))
    const double r = t - rint(t);
    double sn, cs;
    sincospi(2.0 * r, &sn, &cs);
    if (j & 1) {
        cs = -cs;
        sn = -sn;
    }
    if (post && xa) {
        const double re = cs * fp.cre - sn * fp.cim, im = cs * fp.cim + sn * fp.cre;
        cs = re;
        sn = im;
    }
    tabs[i] = make_float2((float)cs, (float)sn);
}

// in and out may be the same plane: every thread reads its elements before the
// transform's first exchange and writes them after the last.
template <int M>
__global__ __launch_bounds__(RowCfg<M>::THREADS) void k_ff_row(const float2* in, float2* out,
                                                              int ny,
                                                              const float2* __restrict__ prex,
                                                              const float2* __restrict__ prey,
                                                              const float2* __restrict__ tw) {
    using C = RowCfg<M>;
    constexpr int E = C::E, T = C::T;
    __shared__ float2 lds[C::RPB * lds_elems<M>()];
    const int sub = threadIdx.x / T, j = threadIdx.x % T;
    const int row = blockIdx.x * C::RPB + sub;
    const bool valid = row < ny;
    const int rr = valid ? row : 0;
    TwCache<M, E> twc;
    twc.load(j, tw);
    const float2 py = prey[rr];
    const float2* src = in + (size_t)rr * M;
    float2 v[1][E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = j + r * T;
        v[0][r] = cmul(src[x], cmul(prex[x], py));
    }
    fft<M, E, 1, FWD>(v, lds + sub * lds_elems<M>(), j, twc);
    if (valid) {
        float2* dst = out + (size_t)row * M;
#pragma unroll
        for (int r = 0; r < E; ++r) dst[j + r * T] = v[0][r];
    }
}

template <int M>
__global__ __launch_bounds__(ColCfg<M>::THREADS) __attribute__((amdgpu_waves_per_eu(ColCfg<M>::WAVES_PER_EU))) void k_ff_col(
    float2* __restrict__ buf, int nx, const float2* __restrict__ postx,
    const float2* __restrict__ posty, const float2* __restrict__ tw) {
    using C = ColCfg<M>;
    constexpr int E = C::E, T = C::T, P = C::P;
    using PK = Pack<float2, P>;
    __shared__ float4 lds4[C::PAIRS * C::LDS_PAIR / 2];
    float2* lds = reinterpret_cast<float2*>(lds4);
    const int pair = threadIdx.x / T, j = threadIdx.x % T;
    const int col0 = (xcd_remap(blockIdx.x, gridDim.x) * C::PAIRS + pair) * P;
    const bool active = col0 < nx;  // blocks may overhang narrow planes (nx is even)
    const int col = active ? col0 : 0;
    float2* base = buf + col;
    TwCache<M, E> twc;
    twc.load(j, tw);
    float2 v[P][E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const PK t = *reinterpret_cast<const PK*>(base + (size_t)(j + r * T) * nx);
#pragma unroll
        for (int p = 0; p < P; ++p) v[p][r] = t.e[p];
    }
    fft<M, E, P, FWD>(v, lds + pair * C::LDS_PAIR, j, twc);
    float2 px[P];
#pragma unroll
    for (int p = 0; p < P; ++p) px[p] = postx[col + p];
    if (!active) return;  // after the last exchange: no barrier follows
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int y = j + r * T;
        const float2 py = posty[y];
        PK t;
#pragma unroll
        for (int p = 0; p < P; ++p) t.e[p] = cmul(v[p][r], cmul(px[p], py));
        *reinterpret_cast<PK*>(base + (size_t)y * nx) = t;
    }
}

hipError_t launch_fresnel_fourier(const float2* in, float2* out, float2* tabs,
                                  const FourierPlan& fp, const float2* twx, const float2* twy,
                                  hipStream_t s) {
    const int len = fp.nx + fp.ny;
    launch_kernel(k_ff_tables, dim3((2 * len + 255) / 256), dim3(256), 0, s, tabs, fp);
    const float2* prex = tabs;
    const float2* prey = tabs + fp.nx;
    const float2* postx = tabs + len;
    const float2* posty = tabs + len + fp.nx;
    CWO_DISPATCH_M(fp.nx, {
        using C = RowCfg<MM>;
        launch_kernel((k_ff_row<MM>), dim3((fp.ny + C::RPB - 1) / C::RPB), dim3(C::THREADS),
                           0, s, in, out, fp.ny, prex, prey, twx);
    });
    CWO_DISPATCH_M(fp.ny, {
        using C = ColCfg<MM>;
        launch_kernel((k_ff_col<MM>), dim3((fp.nx + C::COLS - 1) / C::COLS), dim3(C::THREADS),
                           0, s, out, fp.nx, postx, posty, twy);
    });
    return hipGetLastError();
}

}  // namespace cwo
