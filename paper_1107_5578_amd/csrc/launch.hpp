// Host-side launchers of the diffraction kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace cwo {

// Per-launch FP64 scalars of the angular-spectrum transfer function.
struct AsmScalars {
    double dfx, dfy;  // 1/(Mx dx), 1/(My dy)
    double lam;       // wavelength [m]
    double zl;        // z / wavelength
};

// The angular-spectrum column pass takes the fast phase form when every bin of the
// grid has (lambda fx)^2 + (lambda fy)^2 <= this bound, the exact FP64 form otherwise.
constexpr double kAsmFastMaxS = 0.05;

hipError_t launch_twiddles(float2* tw, int m, hipStream_t s);

// in: batch planes of [ny][nx] (plane stride in_plane elements); out: [ny][mx] per plane
hipError_t launch_row_fwd(const float2* in, float2* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, const float2* tw, hipStream_t s);

// buf: batch planes of [ny][mx], column transform of length my (my = ny or 2*ny)
hipError_t launch_col_asm(float2* buf, int ny, int my, int mx, int batch, size_t plane,
                          const AsmScalars& a, const float2* tw, hipStream_t s);
hipError_t launch_col_fresnel(float2* buf, int ny, int my, int mx, int batch, size_t plane,
                              const float2* hx, const float2* hy, const float2* tw, hipStream_t s);

// in: [ny][mx] per plane; out: [ny][nx] per plane, scaled by `scale`
hipError_t launch_row_inv(const float2* in, float2* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, float scale, const float2* tw,
                          hipStream_t s);

// One axis of the Fresnel transfer function: out[p] = coef * DFT_m(chirp)[p], FP64 inside.
// work must hold 2*m double2.
hipError_t launch_fresnel_axis(double2* work, float2* out, int m, int n, double pitch,
                               double lam_z, double coef_re, double coef_im, hipStream_t s);

}  // namespace cwo
