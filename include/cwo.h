/*
 * cwo.h - C ABI of the MI355X diffraction library (libcwo.so).
 *
 * Scalar diffraction by FFT convolution, as defined in Shimobaba et al.,
 * "Computational wave optics library for C++: CWO++ library" (arXiv 1107.5578):
 *
 *   angular spectrum method (Sec. 2.1.4, Eqs. ang1-ang3):
 *       u2 = IFFT[ FFT[u1] * H_A ],  H_A(fx, fy) = exp(i z sqrt(k^2 - 4 pi^2 (fx^2 + fy^2))),
 *       k = 2 pi / lambda, fx = p * dfx, dfx = 1/(Mx dx) (likewise y);
 *       bins with lambda^2 (fx^2 + fy^2) > 1 are evanescent and get H_A = 0.
 *   Fresnel diffraction, convolution form (Sec. 2.1.1, Eqs. fre_conv, fre_conv_fft,
 *   fre_conv_prop_d):
 *       u2 = C * IFFT[ FFT[u1] * FFT[h_F] ],  h_F(m, n) = exp(i pi/(lambda z) ((m dx)^2 + (n dy)^2)),
 *       C = dx dy exp(i k z) / (i lambda z)  (the quadrature factor dx dy of Eq. fre_conv is kept).
 *
 * Both are convolution forms: the Ny x Nx field is zero-padded to My x Mx = 2Ny x 2Nx, the
 * product spectrum is inverse transformed and the Ny x Nx result is cut out (Sec. 2.1.6),
 * with the field at the top-left of the padded grid. The inverse transform carries
 * 1/(Mx My). Output pitch equals input pitch (Sec. 2.1.1).
 *
 * Data layout: complex64 = interleaved float32 (re, im), row-major [ny][nx], x fastest
 * (the paper's single-precision cwoComplex field). All field pointers are DEVICE pointers
 * owned by the caller; the library never frees them. in == out is allowed.
 *
 * Ordering: cwo_asm / cwo_fresnel / cwo_zstack / cwo_batch are asynchronous and ordered on the
 * given HIP stream (hipStream_t passed as void*, NULL = the null stream); they return
 * after enqueueing. Calls on one context share its scratch memory: serialise them
 * (one stream, or external synchronisation). cwo_submit / cwo_poll are thread-safe.
 *
 * Graph capture: once a call with the same parameters (and, for z-stacks and batches, the
 * same plane count) has run on a context, a propagation call only enqueues kernels on its
 * stream, so it can be captured into a HIP graph and replayed; the first call allocates
 * scratch and tables and must run outside the capture. Profiling must be off. A graph
 * keeps the scratch, table and Fresnel-factor addresses it captured: a later call on the
 * same context that needs more scratch (a larger plane, more planes or points) grows the
 * buffer and frees the old one, and more distinct Fresnel parameter sets than the factor
 * cache holds evict old factors, after which such a graph must not be replayed. Calls
 * that fit the captured sizes, as in a serving loop of fixed shapes, leave it valid.
 *
 * Errors: every call returns a cwo_status. Parameters are validated before anything is
 * launched. A device error makes the context return CWO_ERR_DEVICE from then on.
 * NaN or Inf inside field data is not checked and propagates.
 */
#ifndef CWO_H
#define CWO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CWO_OK = 0,
    CWO_ERR_INVALID = -1,     /* null pointer, non-finite or non-positive pitch/wavelength,
                                 non-finite z, Fresnel with z == 0, unknown kind/flag,
                                 bad count */
    CWO_ERR_UNSUPPORTED = -2, /* size not a power of two in [16, 4096], precision not built
                                 for this call */
    CWO_ERR_NOMEM = -3,       /* device allocation failed, or a job larger than the budget */
    CWO_ERR_DEVICE = -4,      /* a HIP call failed; sticky on the context */
    CWO_ERR_NOTFOUND = -5     /* unknown ticket */
} cwo_status;

/* Diffraction kinds (the paper's CWO_ANGULAR and CWO_FRESNEL_CONV selectors). */
typedef enum {
    CWO_ANGULAR = 1,
    CWO_FRESNEL_CONV = 2,
    CWO_FRESNEL_FOURIER = 3,
    CWO_FRESNEL_SHIFTED = 4
} cwo_kind;

/* Storage precision of the padded intermediate planes; butterflies and the transfer
 * function are always FP32 (phase reduction FP64) and the field in/out is always
 * complex64. FP16/BF16 store each complex as two 16-bit values (round to nearest even);
 * FP16 also scales the field by 2^-e (e = binary exponent of its largest component, found
 * on the device) and every transform by a power of two, undone exactly at the output.
 * Built for cwo_asm / cwo_fresnel (and single jobs of cwo_batch) and cwo_gs in padded
 * mode; elsewhere CWO_ERR_UNSUPPORTED. */
typedef enum { CWO_PREC_F32 = 0, CWO_PREC_F16_STORAGE = 1, CWO_PREC_BF16_STORAGE = 2 } cwo_precision;

/* Flags. CWO_FLAG_NOPAD keeps M = N (circular convolution without padding); it exists for
 * exactness checks such as the plane-wave eigenfunction test, not for production use.
 * CWO_FLAG_FRESNEL_TF (CWO_FRESNEL_CONV only, including z-stacks and batches) multiplies
 * the spectrum by the Fourier transform of the continuous Fresnel kernel (Sec. 2.1.1),
 *     H(fx, fy) = exp(i k z) exp(-i pi lambda z (fx^2 + fy^2)),
 * at the padded grid's frequencies, instead of by C * DFT of the sampled impulse response
 * (the paper's numerical form, the default). The two agree where the sampled chirp is
 * itself band-limited by the grid; elsewhere they are different approximations. Phases
 * are reduced modulo one revolution in FP64. Any other kind with this flag:
 * CWO_ERR_INVALID. */
enum { CWO_FLAG_NOPAD = 1u, CWO_FLAG_FRESNEL_TF = 2u };

typedef struct {
    int32_t nx, ny;      /* field size, each a power of two in [16, 4096]; x is the fastest axis */
    double dx, dy;       /* sampling pitch [m], finite and > 0 (paper default 10e-6) */
    double wavelength;   /* [m], finite and > 0 (paper default 633e-9) */
    double z;            /* propagation distance [m], finite; z < 0 propagates back;
                            z == 0 is the identity for ASM and CWO_ERR_INVALID for Fresnel */
    int32_t kind;        /* cwo_kind; cwo_asm / cwo_fresnel also accept 0 */
    int32_t precision;   /* cwo_precision */
    uint32_t flags;      /* CWO_FLAG_* */
} cwo_params;

/* One propagation request: parameters plus device pointers (caller-owned complex64
 * [ny][nx]). */
typedef struct {
    cwo_params p;
    const void* in;
    void* out;
} cwo_job;

typedef struct cwo_ctx cwo_ctx; /* opaque */

/* Create a context on HIP device `device`. hbm_budget_bytes (0 = no bound) bounds device
 * memory: the workspace of the synchronous calls stays within it (a call that would need
 * more returns CWO_ERR_NOMEM), and the serving scheduler admits a request only while the
 * fields of the admitted, unfinished requests plus everything the context holds (see
 * cwo_memory_held) stay within it. Returns CWO_ERR_INVALID for a null ctx pointer or a bad
 * device ordinal, CWO_ERR_DEVICE if the device cannot be used. */
cwo_status cwo_create(cwo_ctx** ctx, int device, size_t hbm_budget_bytes);

/* Finish every submitted job, wait for all work the context launched, stop its scheduler
 * thread and free its scratch, tables and caches. A null ctx is CWO_ERR_INVALID. */
cwo_status cwo_destroy(cwo_ctx* ctx);

/* Angular spectrum propagation of one field (Sec. 2.1.4, Eq. ang3, padded per Sec. 2.1.6).
 * in, out: device complex64 [ny][nx]. Scratch: ny * 2nx complex64 held by the context. */
cwo_status cwo_asm(cwo_ctx* ctx, const cwo_params* p, const void* in, void* out, void* hip_stream);

/* cwo_asm for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. Same parameters, layout, result
 * (the same kernels, bit for bit) and stream ordering as cwo_asm, but it allocates nothing:
 * its twiddle tables and padded plane live in one statically allocated device array of
 * 64 MiB + 128 KiB that every device the library runs on holds until the process ends.
 * Limits: complex64 storage only (other precisions: CWO_ERR_UNSUPPORTED); the padded plane
 * ny * 2nx complex64 (ny * nx with CWO_FLAG_NOPAD) must fit 64 MiB, i.e. fields up to
 * 2048 x 2048 (larger: CWO_ERR_NOMEM, before any launch). Every call on a device shares that
 * device's array and leaves its contents behind, so calls that overlap on one device (on
 * different streams or from different threads without ordering) race and give wrong
 * results; order them on one stream. */
cwo_status cwo_asm_noalloc(cwo_ctx* ctx, const cwo_params* p, const void* in, void* out,
                           void* hip_stream);

/* Fresnel diffraction, convolution form (Sec. 2.1.1, Eq. fre_conv_fft), same layout as
 * cwo_asm. The two 1-D factors of FFT[h_F] are cached per parameter set. */
cwo_status cwo_fresnel(cwo_ctx* ctx, const cwo_params* p, const void* in, void* out,
                       void* hip_stream);

/* Fresnel diffraction, Fourier form (Sec. 2.1.2, Eqs. fre_fourier1 - fre_fourier3): one
 * unpadded 2-D FFT of the field times exp(i pi (x1^2 + y1^2)/(lambda z)), then times
 * exp(i pi (x2^2 + y2^2)/(lambda z)) and dx dy exp(i k z)/(i lambda z). Sample positions are
 * centred (array index j is coordinate (j - N/2) * pitch) on both planes; the destination
 * pitch is lambda z/(N dx) along x and lambda z/(N dy) along y (negative for z < 0: mirrored
 * axes). in, out: device complex64 [ny][nx]; in == out is allowed. p->kind is 0 or
 * CWO_FRESNEL_FOURIER; z == 0 or any flag is CWO_ERR_INVALID; complex64 storage only
 * (CWO_ERR_UNSUPPORTED otherwise). Scratch: 2 (nx + ny) complex64 of chirp tables. */
cwo_status cwo_fresnel_fourier(cwo_ctx* ctx, const cwo_params* p, const void* in, void* out,
                               void* hip_stream);

/* Destination pitch of cwo_fresnel_fourier for p (host only; validates p the same way). */
cwo_status cwo_fresnel_fourier_pitch(const cwo_params* p, double* dx2, double* dy2);

/* Shifted Fresnel diffraction (Sec. 2.1.3, Eqs. shift_fre1 - shift_fre3): the Fresnel sum
 *   u1[m1, n1] = dx0 dy0 exp(i k z)/(i lambda z)
 *                * sum u0[m0, n0] exp(i pi ((x1 - x0)^2 + (y1 - y0)^2)/(lambda z))
 * from a source window (pitch p->dx, p->dy, centre ox0, oy0) to a destination window of
 * the same size (pitch dx1, dy1, centre ox1, oy1), x0 = m0 dx + ox0, x1 = m1 dx1 + ox1 with
 * centred indices m = j - N/2, computed as a chirp convolution on the 2N x 2N padded grid
 * (3 FFTs, like cwo_fresnel). */
typedef struct {
    double dx1, dy1;  /* destination pitch [m], finite and > 0 */
    double ox0, oy0;  /* source window centre [m] */
    double ox1, oy1;  /* destination window centre [m] */
} cwo_sfresnel;

/* Shifted Fresnel propagation. in, out: device complex64 [ny][nx] (in == out allowed);
 * p->kind is 0 or CWO_FRESNEL_SHIFTED; z == 0, any flag, a null window or a non-finite or
 * non-positive window value is CWO_ERR_INVALID; complex64 storage only. Scratch: ny * 2nx
 * complex64 plus the chirp and kernel-factor tables. */
cwo_status cwo_fresnel_shifted(cwo_ctx* ctx, const cwo_params* p, const cwo_sfresnel* window,
                               const void* in, void* out, void* hip_stream);

/* A propagation whose last pass stores the intensity |u|^2 of the result instead of u
 * (the intensity epilogue of Sec. 3.1 fused into the row inverse store): out is device
 * float [ny][nx], caller-owned, and equals cwo_intensity applied to the output of
 * cwo_asm / cwo_fresnel with the same parameters, bit for bit, without writing or reading
 * the complex result. Parameters, validation, precision and scratch as cwo_asm /
 * cwo_fresnel; out may overlap in (the first pass has consumed in when out is written). */
cwo_status cwo_asm_intensity(cwo_ctx* ctx, const cwo_params* p, const void* in, float* out,
                             void* hip_stream);
cwo_status cwo_fresnel_intensity(cwo_ctx* ctx, const cwo_params* p, const void* in, float* out,
                                 void* hip_stream);

/* Field epilogues of the paper's examples, n elements each, device pointers, ordered on
 * the stream; n == 0 does nothing, a null pointer with n > 0 is CWO_ERR_INVALID.
 *   cwo_intensity: out_f32[i] = re*re + im*im of in_c64[i] (Sec. 3.1), FP32, the two
 *                  products and the sum rounded separately.
 *   cwo_phase:     out_f32[i] = atan2(im, re) in [-pi, pi] (the kinoform, Sec. 7.1).
 *   cwo_polar:     out_c64[i] = a * exp(i phase_f32[i]), a = amp_f32[i] or 1 if amp is
 *                  null (a phase field back to a complex field, Sec. 7.1).
 *   cwo_scale:     (v - min) * (top / (max - min)) over all n values (Sec. 3.1, Eq. norm),
 *                  in FP32 in that order, 0 if max == min; out_u8 = 0 writes float32,
 *                  out_u8 = 1 writes uint8 rounded to nearest (ties to even) and clamped to
 *                  [0, 255] (then top <= 255). top must be finite and > 0. Scratch: a few KiB
 *                  of partial minima and maxima held by the context. */
cwo_status cwo_intensity(cwo_ctx* ctx, const void* in_c64, void* out_f32, size_t n,
                         void* hip_stream);
cwo_status cwo_phase(cwo_ctx* ctx, const void* in_c64, void* out_f32, size_t n, void* hip_stream);
cwo_status cwo_polar(cwo_ctx* ctx, const void* phase_f32, const void* amp_f32, void* out_c64,
                     size_t n, void* hip_stream);
cwo_status cwo_scale(cwo_ctx* ctx, const void* in_f32, void* out, int32_t out_u8, float top,
                     size_t n, void* hip_stream);

/* Shifted angular spectrum method (Sec. 2.1.5, Eqs. shift_ang1 and shift_ang2): the
 * transfer function of cwo_asm times exp(i 2 pi (ox fx + oy fy)) and times the band-limit
 * functions Rect((fx - cx)/wx) Rect((fy - cy)/wy), Rect(t) = 1 for |t| <= 1/2. The linear
 * phase moves the destination window: output sample (m, n) lies at (m dx + ox, n dy + oy)
 * of the unshifted geometry. A width <= 0 leaves that axis unlimited. */
typedef struct {
    double ox, oy; /* destination-window offset [m] */
    double cx, wx; /* band-limit centre and full width along x [1/m] */
    double cy, wy; /* band-limit centre and full width along y [1/m] */
} cwo_shift;

/* Shifted angular spectrum propagation; same layout, scratch and storage precisions as
 * cwo_asm (16-bit storage in the padded form). A null or non-finite shift is
 * CWO_ERR_INVALID. */
cwo_status cwo_asm_shifted(cwo_ctx* ctx, const cwo_params* p, const cwo_shift* shift,
                           const void* in, void* out, void* hip_stream);

/* Band limit of the on-axis case (ox = oy = 0, centred band): sets shift to zero offsets
 * and centres and wx = 2 / (lambda sqrt((2 dfx z)^2 + 1)), dfx = 1/(Mx dx) (M the padded
 * size), wy likewise: the band-limited angular spectrum condition of the reference the
 * section cites, where the transfer function's phase advances by pi per frequency step.
 * Host only; validates p like cwo_asm. */
cwo_status cwo_band_limit(const cwo_params* p, cwo_shift* shift);

/* Schedule of one parameter set, as picked by cwo_autotune. */
typedef struct {
    int32_t row_form;     /* row passes on the row-major plane: 1 a resident grid that
                             prefetches the next rows, 2 one row group per block, 0 the
                             default choice */
    int32_t zchunk;       /* planes per z-stack launch (0: single-plane calls) */
    float us_per_plane;   /* the best measured time */
    int32_t layout;       /* padded plane between the passes: 1 row-major, 2 tiled (four
                             columns per tile, two rows per row-pass group; rows and
                             columns of 8192 as two transforms of 4096), 0 the default
                             choice (tiled for 2048 <= 2nx <= 8192; the Gerchberg-Saxton
                             loop keeps rows of 8192 row-major) */
    int32_t col_form;     /* column pass on the tiled plane, padded columns of 4096 or 8192:
                             1 two adjacent columns per thread, one transform of the full
                             length each; 2 each column as two transforms of half the
                             length (the even and the odd bins), one column per block; 0 the
                             default choice (2 at 8192, 1 at 4096); other planes: 0 only */
} cwo_tuning;

/* Autotuner: runs the candidate schedules of this parameter set (for single planes the
 * plane layout, row-major or tiled where the plane is padded and 2048 <= 2nx <= 8192, the
 * row-pass form of the row-major plane and the column form of the tiled plane; for nz > 1
 * the row-pass form and the z-stack chunk size) on the given buffers, times each on the stream with HIP events (the call
 * synchronises the stream), and keeps the fastest in the context for (kind, nx, ny,
 * precision, flags, nz); later cwo_asm / cwo_fresnel calls (nz = 1) and z-stacks of nz
 * planes with those parameters use it. Results do not depend on the schedule. in:
 * complex64 [ny][nx]; out: complex64 [nz][ny][nx], overwritten; p->z is used for every
 * plane. best may be null. Not thread-safe with other calls on the context.
 * Tune cache: if the environment variable CWO_TUNE_CACHE names a file, cwo_create loads the
 * schedules stored there and each successful cwo_autotune rewrites it with every schedule
 * the context holds (JSON: an array of flat objects, one per line, with the key fields
 * kind, nx, ny, precision, flags, nz and the cwo_tuning fields). An unreadable or missing
 * file is ignored. */
cwo_status cwo_autotune(cwo_ctx* ctx, const cwo_params* p, int32_t nz, const void* in, void* out,
                        void* hip_stream, cwo_tuning* best);

/* Install a schedule for (kind, nx, ny, precision, flags, nz) without timing anything (one
 * chosen elsewhere, e.g. read from a tune cache); a null t removes the context's schedule
 * so the defaults apply again. CWO_ERR_INVALID for out-of-range fields (row_form 0..2,
 * zchunk 0..64, layout 0..2, col_form 0..2), CWO_ERR_UNSUPPORTED for a tiled layout the
 * geometry cannot take or a column form other than 0 where the plane is not tiled with
 * padded columns of 4096 or 8192. Host only; results never depend on the schedule. */
cwo_status cwo_set_tuning(cwo_ctx* ctx, const cwo_params* p, int32_t nz, const cwo_tuning* t);

/* z-stack: one field propagated to nz distances, the paper's 3-D field built by stacking
 * 2-D propagations (Sec. 2.3, Diffract3D). p->kind selects CWO_ANGULAR or
 * CWO_FRESNEL_CONV (0 is CWO_ERR_INVALID here); p->z is ignored; z is a HOST array of nz
 * distances (each validated like p->z). out holds nz planes [nz][ny][nx] complex64 on the
 * device. The row transform of the field and the forward column transforms are done once;
 * planes are processed in chunks of at most 64 that fit the context's budget
 * (CWO_ERR_NOMEM if not even one plane fits). Plane k equals cwo_asm / cwo_fresnel with
 * z = z[k] up to rounding order. p->precision picks the storage of the shared spectrum and
 * of the chunk's planes (complex64, or FP16 / BF16 pairs with the power-of-two scalings of
 * cwo_asm: half the scratch per plane; the padded form only); arithmetic and out stay
 * FP32. */
cwo_status cwo_zstack(cwo_ctx* ctx, const cwo_params* p, const double* z, int32_t nz,
                      const void* in, void* out, void* hip_stream);

/* Batch of independent jobs, stream-ordered, in order. Consecutive jobs on the same input
 * pointer with equal geometry, wavelength, kind, precision and flags are run as one
 * z-stack (their outputs may be anywhere); every other job runs as a single propagation.
 * Each job's p.kind must be CWO_ANGULAR or CWO_FRESNEL_CONV. All jobs are validated before
 * anything is launched. */
cwo_status cwo_batch(cwo_ctx* ctx, const cwo_job* jobs, int32_t njobs, void* hip_stream);

/* Amplitude-constrained ping-pong iteration between two planes a distance p->z apart, by
 * the angular spectrum method (the Gerchberg-Saxton loop of Sec. 7.2 with an amplitude
 * target at both planes; a1 == 1 gives the paper's kinoform variant). One iteration:
 *     v = ASM_{+z}(u);  E_k = || |v| - a2 ||_2 / || a2 ||_2;  v <- a2 v/|v|  (a2 where v == 0)
 *     w = ASM_{-z}(v);  u <- a1 w/|w|  (a1 where w == 0)
 * u: device complex64 [ny][nx], the start field on entry and u after `iterations` steps on
 * exit. a1, a2: device float32 [ny][nx] amplitudes. errors: device float32[iterations]
 * receiving E_k, or NULL. p->kind must be 0 or CWO_ANGULAR. Each propagation is one
 * column pass plus one fused row pass (inverse row FFT, crop, constraint, re-pad,
 * forward row FFT). p->precision picks the storage of the padded spectrum between the
 * passes (complex64, or FP16 / BF16 pairs with the power-of-two scalings of cwo_asm; the
 * FP16 form also scales each field entering a forward transform by 2^-e, e the binary
 * exponent of its largest component: u, then a2 and a1); arithmetic, u and E_k stay
 * FP32 (E_k's sums FP64). Low precision needs the padded form (no CWO_FLAG_NOPAD).
 * Scratch: ny * Mx stored values (Mx = 2nx, or nx with CWO_FLAG_NOPAD), plus
 * iterations * ny * max(1, Mx/1024) + 512 doubles for E_k (the rows' error partials and
 * those of sum(a2^2)). */
cwo_status cwo_gs(cwo_ctx* ctx, const cwo_params* p, const float* a1, const float* a2, void* u,
                  int32_t iterations, float* errors, void* hip_stream);

/* ---- point light sources (Sec. 2.4, Eqs. pls_fre and pls_fre_cgh) ----------------------
 * A 3-D object as N point sources: point j has object coordinates (X_j, Y_j, Z_j) [m] and
 * amplitude A_j, and sits at (ox + X_j, oy + Y_j, oz + Z_j) relative to the hologram's
 * centre; hologram pixel (m, n) is at ((m - nx/2) px, (n - ny/2) py). With
 * r_j^2 = (x - x_j)^2 + (y - y_j)^2 and z_j = oz + Z_j,
 *     cwo_pls_cgh:   I(x, y) = sum_j A_j cos(pi r_j^2/(lambda z_j))            (float out)
 *     cwo_pls_field: u(x, y) = exp(i k oz)/(i lambda oz)
 *                              * sum_j A_j exp(+i pi r_j^2/(lambda z_j))       (complex64 out)
 * (the printed exponent lacks the imaginary unit; the Fresnel wavelet is meant, and the
 * prefactor takes the object's reference distance oz, as the paper's listing sets it).
 * points: device float [npoints][4] records (X, Y, Z, A), 16-byte aligned, read only;
 * npoints == 0 writes zeros. out: device [ny][nx], float (hologram) or complex64 (field),
 * caller-owned. Each term's phase is evaluated and reduced modulo one revolution in FP64,
 * its cosine/sine in FP32; partial sums over 512 points are FP32, the total FP64. Points
 * with z_j == 0 give non-finite values (not checked on the device). Sizes: 1..16384 per
 * axis, any value. Errors, checked in this order: p null -> CWO_ERR_INVALID; sizes out of
 * range -> CWO_ERR_UNSUPPORTED; null pointers, misaligned points, npoints < 0, non-finite
 * or non-positive pitch/wavelength, non-finite offsets or oz == 0 -> CWO_ERR_INVALID.
 * Scratch: 32 bytes per point. Stream-ordered. */
typedef struct {
    int32_t nx, ny;        /* hologram pixels */
    double px, py;         /* hologram pitch [m] */
    double wavelength;     /* [m] */
    double ox, oy, oz;     /* object offset [m]; oz is the reference distance, != 0 */
} cwo_pls_params;

cwo_status cwo_pls_cgh(cwo_ctx* ctx, const cwo_pls_params* p, const float* points,
                       int32_t npoints, float* out, void* hip_stream);
cwo_status cwo_pls_field(cwo_ctx* ctx, const cwo_pls_params* p, const float* points,
                         int32_t npoints, void* out, void* hip_stream);

/* ---- serving (continuous batching) ----------------------------------------------------
 * cwo_submit queues one job and returns at once with a ticket; a scheduler thread of the
 * context admits queued jobs in arrival order when one of its 4 slots (each with its own
 * HIP stream, scratch and Fresnel-factor cache) is free and the job fits the context's HBM
 * budget: the input and output fields of every admitted, unfinished job, all memory the
 * context holds, and what the new batch adds to its slot's scratch together stay within the
 * budget (idle slots free their scratch first when memory is short). A free slot takes the
 * head job and, from the first 256 queued jobs in arrival order, the jobs of its geometry
 * (sizes, pitch, flags, storage) that fit, up to 8 and 512 MiB of padded planes, as one batch
 * on its stream: one launch per pass for the batch (complex64 jobs on one field form a
 * z-stack). A job that shares a buffer with an earlier queued job is not taken ahead of it;
 * every job becomes the head in arrival order (the environment variables
 * CWO_SERVE_MAX_BATCH, CWO_SERVE_WINDOW, CWO_SERVE_BATCH_MIB and CWO_SERVE_POLL_US, read
 * by cwo_create, change the 8 jobs, the window of 256, the 512 MiB and the scheduler's
 * 5 us polling interval while slots run). Requests that arrive while others run are
 * admitted as slots and memory free up, and their work overlaps on the device. Submit and
 * poll never wait for the scheduler's launches or allocations.
 * Footprint of a job (reported by cwo_ticket_info): its input and output fields plus its
 * padded scratch plane (16 nx ny + 8 ny 2nx bytes for complex64 storage). A job larger than
 * the whole budget is rejected with CWO_ERR_NOMEM at submit; one that merely does not fit
 * yet stays queued, and fails with CWO_ERR_NOMEM only if it cannot fit even with every slot
 * idle (memory held by the synchronous calls' workspace).
 * Ordering: cwo_submit does not order the job after any stream, so its input must be
 * complete when it is submitted (e.g. after a synchronisation). cwo_submit_after makes the
 * job's first kernel wait for all work enqueued on hip_stream before the call (an event
 * the library records there), so a field produced by asynchronous kernels on that stream
 * can be submitted at once. The caller keeps in/out alive, and does not touch out, until
 * the ticket reports done. Thread-safe. */

/* Ticket states reported by cwo_poll: 0 queued, 1 running, 2 done, < 0 the job's error. */
typedef struct {
    int32_t state;
    double t_submit, t_start, t_done; /* seconds since cwo_create, host steady clock */
    size_t footprint;                 /* bytes reserved while the job ran */
} cwo_ticket;

cwo_status cwo_submit(cwo_ctx* ctx, const cwo_job* job, uint64_t* ticket);
cwo_status cwo_submit_after(cwo_ctx* ctx, const cwo_job* job, void* hip_stream,
                            uint64_t* ticket);
cwo_status cwo_poll(cwo_ctx* ctx, uint64_t ticket, int32_t* state);
cwo_status cwo_ticket_info(cwo_ctx* ctx, uint64_t ticket, cwo_ticket* info);
/* Forget a finished ticket (CWO_ERR_INVALID while it is queued or running). */
cwo_status cwo_release(cwo_ctx* ctx, uint64_t ticket);
/* Wait until every submitted job has finished; returns the context's sticky status. */
cwo_status cwo_drain(cwo_ctx* ctx);
/* Bytes of device memory the context holds now: twiddle tables, the synchronous calls'
 * workspace and every serving slot's scratch and Fresnel factors (not the caller's fields).
 * Between the scheduler's admissions it stays within the budget. */
cwo_status cwo_memory_held(cwo_ctx* ctx, size_t* bytes);

/* Validate a parameter set for `kind` without touching any device: the same checks the
 * propagation calls run first. Returns CWO_OK, CWO_ERR_INVALID or CWO_ERR_UNSUPPORTED. */
cwo_status cwo_check_params(const cwo_params* p, int32_t kind);

/* Bytes of scratch one propagation of this parameter set needs (0 if the set is invalid). */
size_t cwo_scratch_bytes(const cwo_params* p);

/* Kernel stages, for per-kernel timing. */
typedef enum {
    CWO_STAGE_ROW_FWD = 0,   /* zero-pad + forward row FFT */
    CWO_STAGE_COL = 1,       /* column FFT, transfer function, inverse column FFT, crop */
    CWO_STAGE_ROW_INV = 2,   /* inverse row FFT + crop + 1/(Mx My) */
    CWO_STAGE_TABLES = 3,    /* Fresnel transfer-vector generation */
    CWO_STAGE_COL_Z = 4,     /* z-stack column pass: one forward FFT, per plane H x IFFT */
    CWO_STAGE_ROW_GS = 5,    /* ping-pong row pass: IFFT, crop, constraint, pad, FFT */
    CWO_STAGE_PLS = 6,       /* point-light-source direct sum (with its point pre-pass) */
    CWO_STAGE_COUNT = 8
} cwo_stage;

/* Per-kernel timing for benchmarks. enable != 0 clears the totals and times every stage
 * the context runs afterwards with a pair of HIP events that the runtime stamps from the
 * stage's kernels themselves (the first kernel's start, the last kernel's end; no extra
 * packets enter the stream); 0 stops. cwo_profile_read waits for the recorded events and
 * returns the summed milliseconds and the number of timed launches of one stage. */
cwo_status cwo_profile(cwo_ctx* ctx, int32_t enable);
cwo_status cwo_profile_read(cwo_ctx* ctx, int32_t stage, double* total_ms, int64_t* launches);

/* Human-readable name of a status code (static string, never NULL). */
const char* cwo_strerror(cwo_status s);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t cwo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CWO_H */
