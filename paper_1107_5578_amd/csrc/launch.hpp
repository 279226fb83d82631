// Host-side launchers of the diffraction kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace cwo {

// Stage timing for benchmarks. While a timer is armed on the calling thread, every kernel
// launch of the library stamps the timer's HIP events from the dispatch itself: the first
// kernel of the stage its start, each kernel the stop (so the last one's end stays), and no
// extra packets enter the stream between the kernels.
struct StageTimer {
    hipEvent_t start;
    hipEvent_t stop;
    bool started;  // a kernel has stamped `start`
};
extern thread_local StageTimer* g_stage_timer;

// Per-launch FP64 scalars of the angular-spectrum transfer function.
struct AsmScalars {
    double dfx, dfy;  // 1/(Mx dx), 1/(My dy)
    double lam;       // wavelength [m]
    double zl;        // z / wavelength
};

// Shifted angular spectrum method (Sec. 2.1.5): destination-window offset and the two
// band-limit Rect functions, in the units of the caller's cwo_shift; a width <= 0
// leaves that axis unlimited.
struct AsmShift {
    double ox, oy;  // [m]
    double cx, wx;  // [1/m]
    double cy, wy;  // [1/m]
};

// The angular-spectrum column pass takes the fast phase form when every bin of the
// grid has (lambda fx)^2 + (lambda fy)^2 <= this bound, the exact FP64 form otherwise.
constexpr double kAsmFastMaxS = 0.05;

// Up to this many planes per z-stack launch (per-plane scalars and output pointers
// travel as kernel arguments).
constexpr int kZChunk = 64;

// Per-plane scalars of one z-stack chunk.
struct ZChunk {
    int nz;
    double zl[kZChunk];      // z / lambda of each plane (ASM)
    float2* out[kZChunk];    // destination field of each plane, [ny][nx]
};

// Storage of the padded planes and the power-of-two scalings that keep FP16 in range:
// the field is multiplied by in_scale * (*dyn_scale) before the row transform, the
// transfer function by col_scale, and the output by out_scale * (*dyn_inv).
struct Storage {
    int prec = 0;            // 0 complex64, 1 FP16 pairs, 2 BF16 pairs
    float in_scale = 1.0f;
    const float* dyn_scale = nullptr;
    float col_scale = 1.0f;
    float out_scale = 1.0f;
    const float* dyn_inv = nullptr;
    int row_form = 0;  // row passes: 0 default, 1 persistent with prefetch, 2 one group per block
    int layout = 0;    // padded plane between the passes: 0 row-major, 1 tiled (see tiled_ok)
    int col_form = 0;  // tiled plane, padded columns of 4096 / 8192: 0 default, 1 two columns
                       // per thread at full length, 2 two half-length transforms per column
};

// The tiled plane layout is taken for padded planes (Mx = 2Nx, My = 2Ny) with
// 2048 <= Mx <= 8192 (at Mx = 8192 the row and column passes take the split form: two
// transforms of 4096 per row or column).
inline bool tiled_ok(int nx, int ny, int mx, int my) {
    return mx == 2 * nx && my == 2 * ny && mx >= 2048 && mx <= 8192;
}

constexpr int kRangeBlocks = 1024;
// work[0] = 2^-e, work[1] = 2^e with e = the binary exponent of max(|re|, |im|) over the
// n values; work must hold 2 + kRangeBlocks floats.
hipError_t launch_range_scale(const float2* in, size_t n, float* work, hipStream_t s);
// the same for a real array (e = the exponent of max |a|)
hipError_t launch_range_scale(const float* in, size_t n, float* work, hipStream_t s);

hipError_t launch_twiddles(float2* tw, int m, hipStream_t s);

// precision-generic forms (padded planes only for FP16/BF16)
hipError_t launch_row_fwd(const float2* in, void* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, const Storage& st, const float2* tw,
                          hipStream_t s);
hipError_t launch_col_asm(void* buf, int ny, int my, int mx, int batch, size_t plane,
                          const AsmScalars& a, const Storage& st, const float2* tw, hipStream_t s);
// Column pass of the shifted angular spectrum method, buf in the storage and layout of st;
// masks: mx + my floats of scratch for the band masks.
hipError_t launch_col_asm_shifted(void* buf, int ny, int my, int mx, const AsmScalars& a,
                                  const AsmShift& sh, float* masks, const Storage& st,
                                  const float2* tw, hipStream_t s);
hipError_t launch_col_fresnel(void* buf, int ny, int my, int mx, int batch, size_t plane,
                              const float2* hx, const float2* hy, const Storage& st,
                              const float2* tw, hipStream_t s);
// Column pass of a mixed batch: planes of one geometry in `buf` (plane stride `plane`),
// plane k with the transfer function tf[k]. One call launches the column kernel of one
// form over the planes of that form (none: no launch); complex64, n <= kZChunk.
struct PlaneTF {
    int form;               // 0, 1: ASM fast form, series to s^4 / s^9; 2: ASM exact (not
                            // batched); 3: Fresnel
    float c0;               // fast forms: zl reduced to [-0.5, 0.5]
    double d0, d1, d2, d3;  // fast: lam_dfx, lam_dfy, zl, half_zl; exact: dfx, dfy, lam, zl
    const float2* h;        // Fresnel: Hx (mx entries, with C), then Hy (my entries)
};
hipError_t launch_col_mixed(float2* buf, int ny, int my, int mx, int n, size_t plane,
                            const PlaneTF* tf, int form, const float2* tw, hipStream_t s,
                            int layout);
// The angular-spectrum transfer function a single call takes for these scalars (the fast
// form with its series length, or the exact form).
PlaneTF asm_plane_tf(const AsmScalars& a, int mx, int my);
hipError_t launch_row_inv(const void* in, float2* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, const Storage& st, const float2* tw,
                          hipStream_t s);
// The same for one plane, storing the intensity |u|^2 (float [ny][nx]) instead of u.
hipError_t launch_row_inv_intensity(const void* in, float* out, int nx, int ny, int mx,
                                    const Storage& st, const float2* tw, hipStream_t s);

// in: batch planes of [ny][nx] (plane stride in_plane elements); out: [ny][mx] per plane
hipError_t launch_row_fwd(const float2* in, float2* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, const float2* tw, hipStream_t s,
                          int row_form = 0);

// buf: batch planes of [ny][mx], column transform of length my (my = ny or 2*ny)
hipError_t launch_col_asm(float2* buf, int ny, int my, int mx, int batch, size_t plane,
                          const AsmScalars& a, const float2* tw, hipStream_t s, int layout = 0);


// in: [ny][mx] per plane; out: [ny][nx] per plane, scaled by `scale`
hipError_t launch_row_inv(const float2* in, float2* out, int nx, int ny, int mx, int batch,
                          size_t in_plane, size_t out_plane, float scale, const float2* tw,
                          hipStream_t s);

// z-stack column pass: spec holds the row spectra [ny][mx] of one field (read only);
// for each plane k < zc.nz the column spectrum is multiplied by H(z_k), inverse
// transformed and written to zbuf + k * zplane ([ny][mx] each).
// spec and zbuf hold values in the storage st.prec (padded planes only for 16-bit); the
// stored planes are multiplied by st.col_scale.
hipError_t launch_col_z_asm(const void* spec, void* zbuf, int ny, int my, int mx, size_t zplane,
                            const AsmScalars& a, const ZChunk& zc, const Storage& st,
                            const float2* tw, hipStream_t s);
// Fresnel: the 1-D factors of plane k are at h + k * (mx + my) (Hx with C, then Hy).
hipError_t launch_col_z_fresnel(const void* spec, void* zbuf, int ny, int my, int mx,
                                size_t zplane, const float2* h, int nz, const Storage& st,
                                const float2* tw, hipStream_t s);
// Row inverse of zc.nz planes of zbuf (storage st.prec) into the per-plane outputs
// zc.out[k], multiplied by st.out_scale * (*st.dyn_inv).
hipError_t launch_row_inv_z(const void* zbuf, const ZChunk& zc, int nx, int ny, int mx,
                            size_t zplane, const Storage& st, const float2* tw, hipStream_t s);

// Scalings of the ping-pong row kernel for spectra stored as Storage::prec (0 complex64,
// 1 FP16, 2 BF16): the inverse row transform is multiplied by scale * (*dyn_inv), and
// the constrained field by fwd_scale * (*dyn_fwd) before the forward transform; null
// dyn pointers count as 1.
struct GsScale {
    int prec = 0;
    float scale = 1.0f;
    const float* dyn_inv = nullptr;
    float fwd_scale = 1.0f;
    const float* dyn_fwd = nullptr;
    int layout = 0;  // layout of spec: 0 row-major, 1 tiled
};
// Ping-pong iteration row kernel. For each of the ny rows of spec ([ny][mx] in the
// storage of gsc.prec, the output of a column pass): inverse row FFT, keep the first nx
// values scaled as gsc says, replace each value u by a*u/|u| (a where u == 0) with a from
// amp ([ny][nx] float32), and, if num is not null, store the row's FP64 sum of
// (|u| - a)^2 as P = gs_partials(mx) partials at num[row*P .. row*P + P-1]. Then either
// (out == nullptr) zero-pad and forward row FFT back into spec, or write the constrained
// field to out ([ny][nx] complex64).
hipError_t launch_row_gs(void* spec, const float* amp, float2* out, double* num, int nx, int ny,
                         int mx, const GsScale& gsc, const float2* tw, hipStream_t s);
int gs_partials(int mx);
// errors[k] = sqrt(sum of num[k*ny*P ..] over the ny*P partials / sum(amp^2)), k < iters,
// P = gs_partials(mx); den_work holds kGsDenParts doubles (the denominator's partials).
constexpr int kGsDenParts = 512;
hipError_t launch_gs_errors(const double* num, const float* amp, double* den_work, float* errors,
                            int nx, int ny, int mx, int iters, hipStream_t s);

// Fresnel transfer-function factors of up to kZChunk planes that share the geometry:
// plane k gets Hx_k = C_k * DFT_mx(hx_k) at out + k*(mx+my) and Hy_k = DFT_my(hy_k) right
// after it, where h*_k are the sampled 1-D chirps exp(i pi (s(d) pitch)^2 / (lambda z_k)).
// With `analytic` set, the factors are instead the two halves of the Fourier transform of
// the continuous Fresnel kernel: Hx_k = C_k exp(-i pi lambda z_k fx^2), Hy_k =
// exp(-i pi lambda z_k fy^2) at the padded grid's frequencies.
struct FresnelPlanes {
    int mx, nx, my, ny;
    double dx, dy;
    int nz;
    int analytic;                 // 0: DFT of the sampled chirps, 1: analytic factors
    double inv2lz[kZChunk];       // 1 / (2 lambda z_k): chirp phase in revolutions per m^2
    double hlz[kZChunk];          // lambda z_k / 2: analytic phase in revolutions per (1/m)^2
    double cre[kZChunk], cim[kZChunk];  // C_k: dx dy exp(i k z_k) / (i lambda z_k), or
                                        // exp(i k z_k) for the analytic factors
};
// work must hold mx + my double2 (the FP64 twiddle tables; unused by the analytic
// factors); mx, my <= 8192.
hipError_t launch_fresnel_planes(double2* work, float2* out, const FresnelPlanes& fp,
                                 hipStream_t s);

// Point-light-source sums (hologram or field) over npts points given as float
// (X, Y, Z, A) records (16-byte aligned); work holds pls_work_bytes(npts). The hologram
// pixel (m, n) sits at ((m - nx/2) px, (n - ny/2) py); point j at (ox + X, oy + Y,
// oz + Z). The field is multiplied by (cre, cim).
struct PlsParams {
    int nx, ny;
    double px, py, lam;
    double ox, oy, oz;
    double cre, cim;
};
hipError_t launch_pls(const float* points, int npts, void* work, void* out, bool field,
                      const PlsParams& pp, hipStream_t s);
size_t pls_work_bytes(int npts);

// Independent fields of one geometry in one launch per pass: the row forward pass reads
// plane k from ins.in[k] into scratch plane k, the row inverse writes plane k to
// outs.out[k] (batch <= kZChunk; complex64).
// Plane addressing: equally spaced planes, or one pointer per plane (input of the row
// forward pass, output of the row inverse).
struct InStrided {
    const float2* in;
    size_t plane;
    __device__ __forceinline__ const float2* operator()(int k) const { return in + k * plane; }
};
struct InTable {
    const float2* in[kZChunk];
    __device__ __forceinline__ const float2* operator()(int k) const { return in[k]; }
};

// Output of the row inverse passes: put(k, i, v) stores value v of element i (row-major
// [ny][nx] index) of plane k.
struct OutStrided {
    float2* out;
    size_t plane;
    __device__ __forceinline__ void put(int k, size_t i, float2 v) const { out[k * plane + i] = v; }
};
struct OutTable {
    float2* out[kZChunk];
    __device__ __forceinline__ void put(int k, size_t i, float2 v) const { out[k][i] = v; }
};
// The intensity |v|^2 instead of the field (Sec. 3.1), each product and the sum rounded
// on its own in FP32 (no fused multiply-add), so it equals the intensity of the stored field.
struct OutIntensity {
    float* out;
    size_t plane;
    __device__ __forceinline__ void put(int k, size_t i, float2 v) const {
#pragma clang fp contract(off)
        out[k * plane + i] = v.x * v.x + v.y * v.y;
    }
};
hipError_t launch_row_fwd_tab(const InTable& ins, float2* out, int nx, int ny, int mx, int batch,
                              size_t out_plane, const float2* tw, hipStream_t s, int layout = 0);
hipError_t launch_row_inv_tab(const float2* in, const OutTable& outs, int nx, int ny, int mx,
                              int batch, size_t in_plane, float scale, const float2* tw,
                              hipStream_t s, int layout = 0);

// Fresnel diffraction in Fourier form (Sec. 2.1.2): parameters of the chirp tables.
struct FourierPlan {
    int nx, ny;
    double dx, dy;    // source pitch [m]
    double dx2, dy2;  // destination pitch lambda z/(N d) [m]
    double inv2lz;    // 1/(2 lambda z)
    double cre, cim;  // dx dy exp(i k z)/(i lambda z)
};
// in, out: complex64 [ny][nx] (may alias); tabs: 2 (nx + ny) complex64 of scratch;
// twx, twy: twiddle tables of length nx and ny.
hipError_t launch_fresnel_fourier(const float2* in, float2* out, float2* tabs,
                                  const FourierPlan& fp, const float2* twx, const float2* twy,
                                  hipStream_t s);

// Shifted Fresnel diffraction (Sec. 2.1.3): parameters of the source and destination
// chirp tables.
struct SfPlan {
    int nx, ny;
    double px0, py0, px1, py1;  // source and destination pitch [m]
    double ox0, oy0, ox1, oy1;  // window centres [m]
    double inv_lz;              // 1/(lambda z)
    double cre, cim;            // dx0 dy0 exp(i k z)/(i lambda z)
};
// tabs: 2 (nx + ny) complex64 (source chirps, then destination chirps with the constant).
hipError_t launch_sf_tables(float2* tabs, const SfPlan& sp, hipStream_t s);
// Padded row forward of the chirped field into scratch [ny][2nx].
hipError_t launch_sf_row_fwd(const float2* in, float2* out, int nx, int ny, const float2* tabs,
                             const float2* tw, hipStream_t s);
// Row inverse of scratch [ny][2nx], crop, scale and destination chirp into out [ny][nx].
hipError_t launch_sf_row_inv(const float2* in, float2* out, int nx, int ny, float scale,
                             const float2* tabs, const float2* tw, hipStream_t s);

// Field epilogues (Sec. 3.1, Sec. 7.1). launch_scale needs work of 4 + 2 * kRangeBlocks
// floats (min, max and the factor first, then per-block partials).
hipError_t launch_intensity(const float2* in, float* out, size_t n, hipStream_t s);
hipError_t launch_phase(const float2* in, float* out, size_t n, hipStream_t s);
hipError_t launch_polar(const float* phi, const float* amp, float2* out, size_t n, hipStream_t s);
hipError_t launch_scale(const float* in, size_t n, float top, bool u8, void* out, float* work,
                        hipStream_t s);

}  // namespace cwo
