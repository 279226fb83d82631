/*
 * Oracle: textbook FP64 complex FFT (test infrastructure only).
 *
 * This file belongs to the CPU reference used by the tests, the smoke check and
 * the CPU baseline of the benchmark. The product library never links it, and it
 * includes no header of the product.
 *
 * What it computes: the discrete Fourier transform
 *     X[k] = sum_{j=0}^{M-1} x[j] * exp(s * 2*pi*i * j*k / M),   s = -1 forward, +1 inverse,
 * unnormalised in both directions (the 1/M factor of the inverse is applied by
 * the caller, where the diffraction oracle writes its inverse step out). The
 * paper uses the FFT as the fast route to this map for its `FFT`/`IFFT`
 * primitives (Sec. 3, the virtual primitives of the CWO/GWO classes).
 *
 * Algorithm: iterative radix-2 decimation-in-time Cooley-Tukey on a power-of-two
 * length, bit-reversal permutation first, then log2(M) butterfly levels. The
 * twiddles exp(-2*pi*i*k/M), k < M/2, come from a table built with the C library's
 * cos/sin of the exact FP64 argument 2*pi*k/M folded into the first octant, so
 * each entry is correctly rounded to within an ulp. Nothing is blocked or fused.
 *
 * The 2-D transform applies the 1-D transform to every row, then to every column
 * (separability of the 2-D DFT). OpenMP spreads rows/columns over host threads;
 * each row/column is transformed exactly as in the serial code, so results do
 * not depend on the thread count.
 *
 * Layout: interleaved complex128 (re, im), row-major [ny][nx], i.e. numpy complex128.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } c128;

static int is_pow2(int64_t m) { return m > 0 && (m & (m - 1)) == 0; }

/* exp(-2*pi*i*k/m) for 0 <= k < m, using symmetry so the libm argument stays in [0, pi/4]. */
static c128 twiddle(int64_t k, int64_t m) {
    /* angle = 2*pi*k/m; reduce k into octants of the circle exactly in integers */
    const double two_pi = 6.283185307179586476925286766559;
    int64_t k8 = k * 8;          /* angle in units of (2*pi/8)/m */
    int64_t oct = k8 / m;        /* which octant, 0..7 */
    int64_t rem = k8 - oct * m;  /* remainder in units of (2*pi/8)/m, 0 <= rem < m */
    double a;                    /* angle inside the octant, [0, pi/4) */
    double c, s;                 /* cos, sin of the full angle */
    /* mirror odd octants so the libm argument is within [0, pi/4] */
    int mirror = (int)(oct & 1);
    int64_t r = mirror ? (m - rem) : rem;
    a = (two_pi / 8.0) * ((double)r / (double)m);
    double ca = cos(a), sa = sin(a);
    /* base angle of octant 'oct' is oct*pi/4; for mirrored octants the angle is (oct+1)*pi/4 - a */
    switch (oct) {
        case 0: c = ca;  s = sa;  break;   /* a */
        case 1: c = sa;  s = ca;  break;   /* pi/2 - a */
        case 2: c = -sa; s = ca;  break;   /* pi/2 + a */
        case 3: c = -ca; s = sa;  break;   /* pi - a */
        case 4: c = -ca; s = -sa; break;   /* pi + a */
        case 5: c = -sa; s = -ca; break;   /* 3pi/2 - a */
        case 6: c = sa;  s = -ca; break;   /* 3pi/2 + a */
        default: c = ca; s = -sa; break;   /* 2pi - a */
    }
    c128 w = { c, -s };  /* exp(-i*angle) */
    return w;
}

static void fft1d(c128* x, int64_t m, int64_t stride, const c128* tw, int inverse, c128* buf) {
    /* gather (strided) into buf in bit-reversed order */
    int levels = 0;
    while (((int64_t)1 << levels) < m) ++levels;
    for (int64_t i = 0; i < m; ++i) {
        int64_t r = 0, v = i;
        for (int b = 0; b < levels; ++b) { r = (r << 1) | (v & 1); v >>= 1; }
        buf[r] = x[i * stride];
    }
    /* butterfly levels: sub-transform size 'len' doubles each level */
    for (int64_t len = 2; len <= m; len <<= 1) {
        int64_t half = len / 2;
        int64_t tstep = m / len;            /* twiddle index step in the size-m table */
        for (int64_t base = 0; base < m; base += len) {
            for (int64_t k = 0; k < half; ++k) {
                c128 w = tw[k * tstep];
                if (inverse) w.im = -w.im;
                c128 a = buf[base + k];
                c128 b = buf[base + k + half];
                c128 t = { b.re * w.re - b.im * w.im, b.re * w.im + b.im * w.re };
                buf[base + k].re = a.re + t.re;
                buf[base + k].im = a.im + t.im;
                buf[base + k + half].re = a.re - t.re;
                buf[base + k + half].im = a.im - t.im;
            }
        }
    }
    for (int64_t i = 0; i < m; ++i) x[i * stride] = buf[i];
}

static c128* make_table(int64_t m) {
    c128* tw = (c128*)malloc(sizeof(c128) * (size_t)(m / 2 > 0 ? m / 2 : 1));
    for (int64_t k = 0; k < m / 2; ++k) tw[k] = twiddle(k, m);
    return tw;
}

/* 1-D transform of one contiguous vector; returns 0 on success, -1 on bad size. */
int oracle_fft1(double* data, int64_t m, int inverse) {
    if (!is_pow2(m)) return -1;
    c128* tw = make_table(m);
    c128* buf = (c128*)malloc(sizeof(c128) * (size_t)m);
    fft1d((c128*)data, m, 1, tw, inverse, buf);
    free(buf);
    free(tw);
    return 0;
}

/* The twiddle table entry exp(-2*pi*i*k/m), exposed so tests can pin it. */
void oracle_twiddle(int64_t k, int64_t m, double* out2) {
    c128 w = twiddle(k, m);
    out2[0] = w.re;
    out2[1] = w.im;
}

/* 2-D transform of a row-major [ny][nx] array: rows, then columns. */
int oracle_fft2(double* data, int64_t ny, int64_t nx, int inverse, int nthreads) {
    if (!is_pow2(nx) || !is_pow2(ny)) return -1;
    c128* x = (c128*)data;
    c128* twx = make_table(nx);
    c128* twy = make_table(ny);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        c128* buf = (c128*)malloc(sizeof(c128) * (size_t)(nx > ny ? nx : ny));
#pragma omp for schedule(static)
        for (int64_t r = 0; r < ny; ++r) fft1d(x + r * nx, nx, 1, twx, inverse, buf);
#pragma omp for schedule(static)
        for (int64_t c = 0; c < nx; ++c) fft1d(x + c, ny, nx, twy, inverse, buf);
        free(buf);
    }
    free(twx);
    free(twy);
    return 0;
}

/* Number of threads an OpenMP region would use (for reporting the CPU baseline). */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
