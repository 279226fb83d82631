// Shifted Fresnel diffraction (Sec. 2.1.3, Eqs. shift_fre1 - shift_fre3): the Fresnel sum
// between a source window (pitch p0, centre O0) and a destination window (pitch p1,
// centre O1) as a chirp convolution. Per axis, with centred indices m and
// x0 = m0 p0 + O0, x1 = m1 p1 + O1, S = p0 p1/(lambda z):
//     (x1 - x0)^2/(lambda z) = x0^2/(lambda z) - 2 m0 p0 O1/(lambda z) - S m0^2
//                            + S (m1 - m0)^2
//                            + x1^2/(lambda z) - 2 (m1 p1 O0 + O1 O0)/(lambda z) - S m1^2,
// so the field is multiplied by the source chirp (first line), convolved with
// h(d) = exp(i pi S d^2) on the 2N x 2N padded grid (the Fresnel convolution pass, whose
// factor tables take the chirp pitch sqrt(p0 p1)), and multiplied by the destination
// chirp (last line) and dx0 dy0 exp(i k z)/(i lambda z) when stored.

#include "kernel_common.hpp"

namespace cwo {

// tabs = [prex (nx) | prey (ny) | postx (nx, with the constant) | posty (ny)]; phases in
// revolutions in FP64, reduced modulo one before the sine and cosine.
__global__ void k_sf_tables(float2* __restrict__ tabs, SfPlan sp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int len = sp.nx + sp.ny;
    if (i >= 2 * len) return;
    const bool post = i >= len;
    const int k = post ? i - len : i;
    const bool xa = k < sp.nx;
    const int j = xa ? k : k - sp.nx;
    const int n = xa ? sp.nx : sp.ny;
    const double p0 = xa ? sp.px0 : sp.py0, p1 = xa ? sp.px1 : sp.py1;
    const double o0 = xa ? sp.ox0 : sp.oy0, o1 = xa ? sp.ox1 : sp.oy1;
    const double m = (double)(j - n / 2);
    const double s = p0 * p1 * sp.inv_lz;
    double t;
    if (!post) {
        const double x0 = m * p0 + o0;
        t = x0 * x0 * (0.5 * sp.inv_lz) - m * p0 * o1 * sp.inv_lz - 0.5 * s * m * m;
    } else {
        const double x1 = m * p1 + o1;
        t = x1 * x1 * (0.5 * sp.inv_lz) - (m * p1 * o0 + o1 * o0) * sp.inv_lz - 0.5 * s * m * m;
    }
    const double r = t - rint(t);
    double sn, cs;
    sincospi(2.0 * r, &sn, &cs);
    if (post && xa) {
        const double re = cs * sp.cre - sn * sp.cim, im = cs * sp.cim + sn * sp.cre;
        cs = re;
        sn = im;
    }
    tabs[i] = make_float2((float)cs, (float)sn);
}

// Row forward of the padded plane: nx values times the source chirp, zeros beyond.
template <int M>
__global__ __launch_bounds__(RowCfg<M>::THREADS) void k_sf_row_fwd(
    const float2* __restrict__ in, float2* __restrict__ out, int nx, int ny,
    const float2* __restrict__ prex, const float2* __restrict__ prey,
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
    const float2* src = in + (size_t)rr * nx;
    float2 v[1][E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int x = j + r * T;
        v[0][r] = (r < E / 2) ? cmul(src[x], cmul(prex[x], py)) : make_float2(0.f, 0.f);
    }
    fft<M, E, 1, FWD>(v, lds + sub * lds_elems<M>(), j, twc);
    if (valid) {
        float2* dst = out + (size_t)row * M;
#pragma unroll
        for (int r = 0; r < E; ++r) dst[j + r * T] = v[0][r];
    }
}

// Row inverse with the crop to nx, the 1/(Mx My) scale and the destination chirp.
template <int M>
__global__ __launch_bounds__(RowCfg<M>::THREADS) void k_sf_row_inv(
    const float2* __restrict__ in, float2* __restrict__ out, int nx, int ny, float scale,
    const float2* __restrict__ postx, const float2* __restrict__ posty,
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
    const float2* src = in + (size_t)rr * M;
    float2 v[1][E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[0][r] = src[j + r * T];
    fft<M, E, 1, INV>(v, lds + sub * lds_elems<M>(), j, twc);
    if (!valid) return;
    const float2 py = posty[row];
    float2* dst = out + (size_t)row * nx;
#pragma unroll
    for (int r = 0; r < E / 2; ++r) {
        const int x = j + r * T;
        const float2 w = make_float2(v[0][r].x * scale, v[0][r].y * scale);
        dst[x] = cmul(w, cmul(postx[x], py));
    }
}

hipError_t launch_sf_tables(float2* tabs, const SfPlan& sp, hipStream_t s) {
    const int len = sp.nx + sp.ny;
    launch_kernel(k_sf_tables, dim3((2 * len + 255) / 256), dim3(256), 0, s, tabs, sp);
    return hipGetLastError();
}

hipError_t launch_sf_row_fwd(const float2* in, float2* out, int nx, int ny, const float2* tabs,
                             const float2* tw, hipStream_t s) {
    const int mx = 2 * nx;
    CWO_DISPATCH_M(mx, {
        using C = RowCfg<MM>;
        launch_kernel((k_sf_row_fwd<MM>), dim3((ny + C::RPB - 1) / C::RPB), dim3(C::THREADS),
                           0, s, in, out, nx, ny, tabs, tabs + nx, tw);
    });
    return hipGetLastError();
}

hipError_t launch_sf_row_inv(const float2* in, float2* out, int nx, int ny, float scale,
                             const float2* tabs, const float2* tw, hipStream_t s) {
    const int mx = 2 * nx;
    const float2* postx = tabs + nx + ny;
    const float2* posty = postx + nx;
    CWO_DISPATCH_M(mx, {
        using C = RowCfg<MM>;
        launch_kernel((k_sf_row_inv<MM>), dim3((ny + C::RPB - 1) / C::RPB), dim3(C::THREADS),
                           0, s, in, out, nx, ny, scale, postx, posty, tw);
    });
    return hipGetLastError();
}

}  // namespace cwo
