// Device-side FFT building blocks for gfx950 (wave64, LDS-staged Stockham).
//
// A length-M transform is done by one group of T = M/E threads; each thread
// holds E complex values in registers. Before every pass thread j holds the
// elements j + r*T (r < E) of the current sequence; a radix-RP pass performs
// E/RP butterflies b = j + i*T, each reading inputs b + kk*(M/RP), multiplying
// by the Stockham twiddle W_{Ns*RP}^{(b mod Ns)*kk} and writing outputs to
// (b / Ns)*Ns*RP + (b mod Ns) + kk*Ns, where Ns is the product of the radices
// of the earlier passes. Intermediate passes exchange through LDS; the first
// pass reads registers loaded straight from global memory and the last pass
// leaves the result in registers in natural order (element j + r*T), so global
// loads and stores are both unit-stride across a wavefront.
//
// Sign convention: forward uses exp(-2*pi*i*jk/M), inverse exp(+2*pi*i*jk/M),
// both unnormalised (the DFT pair the paper's FFT/IFFT primitives compute).
#pragma once
#include <hip/hip_runtime.h>

namespace cwo {

constexpr int FWD = -1;
constexpr int INV = +1;

// ---- storage of the padded intermediate planes --------------------------------
// complex64 (FP32), or two FP16 / two BF16 values per complex (rounded to nearest
// even on the way in). Arithmetic is always FP32.
struct StF32 {
    using E = float2;
    __device__ __forceinline__ static float2 dec(E v) { return v; }
    __device__ __forceinline__ static E enc(float2 v) { return v; }
};
struct alignas(4) half2s {
    _Float16 x, y;
};
struct StF16 {
    using E = half2s;
    __device__ __forceinline__ static float2 dec(E v) { return make_float2((float)v.x, (float)v.y); }
    __device__ __forceinline__ static E enc(float2 v) { return E{(_Float16)v.x, (_Float16)v.y}; }
};
struct alignas(4) bf162s {
    __bf16 x, y;
};
struct StBF16 {
    using E = bf162s;
    __device__ __forceinline__ static float2 dec(E v) { return make_float2((float)v.x, (float)v.y); }
    __device__ __forceinline__ static E enc(float2 v) { return E{(__bf16)v.x, (__bf16)v.y}; }
};
// P adjacent stored elements, loaded and stored as one vector access
template <class E, int P>
struct alignas(sizeof(E) * P) Pack {
    E e[P];
};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(__fmaf_rn(a.x, b.x, -a.y * b.y), __fmaf_rn(a.x, b.y, a.y * b.x));
}
// multiply by w (DIR = FWD) or conj(w) (DIR = INV); tables store exp(-2*pi*i*k/M)
template <int DIR>
__device__ __forceinline__ float2 ctw(float2 a, float2 w) {
    if constexpr (DIR == FWD) return cmul(a, w);
    else return make_float2(__fmaf_rn(a.x, w.x, a.y * w.y), __fmaf_rn(a.y, w.x, -a.x * w.y));
}
// multiply by exp(DIR * i*pi/2): -i forward, +i inverse
template <int DIR>
__device__ __forceinline__ float2 rot90(float2 a) {
    if constexpr (DIR == FWD) return make_float2(a.y, -a.x);
    else return make_float2(-a.y, a.x);
}

// Multiply by exp(DIR * 2*pi*i*m/R) for a compile-time m, cheap forms for multiples of pi/4.
template <int R, int M_, int DIR>
__device__ __forceinline__ float2 wconst(float2 a) {
    constexpr int m = ((M_ % R) + R) % R;
    if constexpr (m == 0) return a;
    else if constexpr (8 * m % R == 0) {
        constexpr int oct = 8 * m / R;  // angle = oct * pi/4
        constexpr float h = 0.70710678118654752440f;
        if constexpr (oct == 2) return rot90<DIR>(a);
        else if constexpr (oct == 4) return make_float2(-a.x, -a.y);
        else if constexpr (oct == 6) return rot90<-DIR>(a);
        else {
            // (+-1 +- i)/sqrt(2): angle = DIR*oct*pi/4
            constexpr float c = (oct == 1 || oct == 7) ? h : -h;
            constexpr float s0 = (oct == 1 || oct == 3) ? h : -h;  // sin(oct*pi/4)
            constexpr float s = (DIR == FWD) ? -s0 : s0;
            // fused as in the general case, so that every kernel rounds it alike
            return make_float2(__fmaf_rn(c, a.x, -s * a.y), __fmaf_rn(c, a.y, s * a.x));
        }
    } else {
        // general angle 2*pi*m/R with R <= 32: cos/sin of multiples of pi/16
        constexpr double PI = 3.14159265358979323846;
        // constexpr evaluation through a small table of cos(k*pi/16), k = 0..8
        constexpr double ctab[9] = {1.0, 0.98078528040323044913, 0.92387953251128675613,
                                    0.83146961230254523708, 0.70710678118654752440,
                                    0.55557023301960222474, 0.38268343236508977173,
                                    0.19509032201612826785, 0.0};
        constexpr int k32 = m * (32 / R);  // angle in units of pi/16, 0..31
        constexpr int q = k32 / 8, rr = k32 % 8;
        // cos and sin of (q*pi/2 + rr*pi/16)
        constexpr double c0 = ctab[rr], s0 = ctab[8 - rr];
        constexpr double cc = q == 0 ? c0 : q == 1 ? -s0 : q == 2 ? -c0 : s0;
        constexpr double ss = q == 0 ? s0 : q == 1 ? c0 : q == 2 ? -s0 : -c0;
        constexpr float c = (float)cc;
        constexpr float s = (float)(DIR == FWD ? -ss : ss);
        (void)PI;
        return make_float2(__fmaf_rn(c, a.x, -s * a.y), __fmaf_rn(c, a.y, s * a.x));
    }
}

// ---- small DFTs on register arrays, in place, natural output order ------------

template <int DIR>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
    float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
    float2 t2 = cadd(a1, a3), t3 = rot90<DIR>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// DFT of 4 points of which the last two are zero: 8 additions instead of 16.
template <int DIR>
__device__ __forceinline__ void dft4_zin(float2& a0, float2& a1, float2& a2, float2& a3) {
    const float2 x0 = a0, x1 = a1, r = rot90<DIR>(a1);
    a0 = cadd(x0, x1);
    a2 = csub(x0, x1);
    a1 = cadd(x0, r);
    a3 = csub(x0, r);
}

// DFT of R points held in v[OFF + STRIDE*k], k < R, result in the same slots in natural order.
// ZIN: the inputs k >= R/2 are known to be zero (the zero-padded half of a transform's
// first pass) and are neither read nor added; each half-size DFT of the decimation in
// time then has a zero upper half as well.
template <int R, int DIR, int OFF = 0, int STRIDE = 1, bool ZIN = false, int N>
__device__ __forceinline__ void dft(float2 (&v)[N]) {
    static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 16 || R == 32, "radix");
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        if constexpr (ZIN) v[OFF + STRIDE] = v[OFF];
        else dft2<DIR>(v[OFF], v[OFF + STRIDE]);
    } else if constexpr (R == 4) {
        if constexpr (ZIN) dft4_zin<DIR>(v[OFF], v[OFF + STRIDE], v[OFF + 2 * STRIDE], v[OFF + 3 * STRIDE]);
        else dft4<DIR>(v[OFF], v[OFF + STRIDE], v[OFF + 2 * STRIDE], v[OFF + 3 * STRIDE]);
    } else if constexpr (R == 8 || R == 32) {
        // radix-2 decimation in time over two half-size DFTs
        constexpr int H = R / 2;
        dft<H, DIR, OFF, 2 * STRIDE, ZIN>(v);           // even samples
        dft<H, DIR, OFF + STRIDE, 2 * STRIDE, ZIN>(v);  // odd samples
        float2 t[R];
#pragma unroll
        for (int k = 0; k < R; ++k) t[k] = v[OFF + k * STRIDE];
        // t[2k] = E[k], t[2k+1] = O[k]
        float2 o[R];
        [&]<int... K>(std::integer_sequence<int, K...>) {
            ((o[K] = cadd(t[2 * K], wconst<R, K, DIR>(t[2 * K + 1])),
              o[K + H] = csub(t[2 * K], wconst<R, K, DIR>(t[2 * K + 1]))), ...);
        }(std::make_integer_sequence<int, H>{});
#pragma unroll
        for (int k = 0; k < R; ++k) v[OFF + k * STRIDE] = o[k];
    } else {  // R == 16: 4 x 4
        // stage 1: for each n2, DFT4 over n1 of x[4*n1 + n2]; result Y[n2][k1] kept at slot 4*k1 + n2
        // (with ZIN, x[4*n1 + n2] = 0 for n1 >= 2)
        dft<4, DIR, OFF + 0 * STRIDE, 4 * STRIDE, ZIN>(v);
        dft<4, DIR, OFF + 1 * STRIDE, 4 * STRIDE, ZIN>(v);
        dft<4, DIR, OFF + 2 * STRIDE, 4 * STRIDE, ZIN>(v);
        dft<4, DIR, OFF + 3 * STRIDE, 4 * STRIDE, ZIN>(v);
        // twiddles W16^(n2*k1) on slot 4*k1 + n2
        float2 y[16];
        [&]<int... S>(std::integer_sequence<int, S...>) {
            ((y[S] = wconst<16, (S % 4) * (S / 4), DIR>(v[OFF + S * STRIDE])), ...);
        }(std::make_integer_sequence<int, 16>{});
        // stage 2: for each k1, DFT4 over n2 of Y[n2][k1] -> X[k1 + 4*k2]
        dft4<DIR>(y[0], y[1], y[2], y[3]);
        dft4<DIR>(y[4], y[5], y[6], y[7]);
        dft4<DIR>(y[8], y[9], y[10], y[11]);
        dft4<DIR>(y[12], y[13], y[14], y[15]);
        // y[4*k1 + k2] = X[k1 + 4*k2]
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[OFF + (k1 + 4 * k2) * STRIDE] = y[4 * k1 + k2];
    }
}

// ---- pass plans -------------------------------------------------------------

// Radix of pass p for a length-M transform with E values per thread: the first
// pass takes the remainder M / E^(P-1), the others take E (E itself may be 32,
// then later passes use 16 and each thread runs two butterflies).
template <int M, int E>
struct Plan {
    static constexpr int log2i(int x) { return x <= 1 ? 0 : 1 + log2i(x / 2); }
    static constexpr int LM = log2i(M);
    static constexpr int LR = (E == 32) ? 4 : log2i(E);  // bits per full pass
    static constexpr int LE = log2i(E);
    // E == 32: first pass radix 32 (if it fits), the rest radix 16
    static constexpr int FIRST_BITS =
        (E == 32) ? LE : ((LM % LR) == 0 ? LR : (LM % LR));
    static constexpr int REST = (LM - FIRST_BITS) / LR;
    static constexpr int PASSES = 1 + REST;
    static constexpr int T = M / E;
    static_assert((E == 32 ? (LM - LE) % 4 == 0 : true), "E=32 plans need M = 32 * 16^k");
    static constexpr int radix(int p) { return p == 0 ? (1 << FIRST_BITS) : (1 << LR); }
    static constexpr int ns(int p) { return p == 0 ? 1 : (1 << FIRST_BITS) << (LR * (p - 1)); }
};

// Twiddles of every pass for one thread, loaded once (they depend on the thread index
// only): W_{Ns*RP}^{(b mod Ns)*kk} for each butterfly b = j + i*T and kk = 1..RP-1,
// stored at w[pass][i*RP + kk]. Loading them up front takes the twiddle loads off the
// critical path between LDS exchanges, and a forward and an inverse transform of the
// same length share them (the inverse conjugates on use).
template <int M, int E>
struct TwCache {
    using PL = Plan<M, E>;
    float2 w[PL::PASSES][E];
    // tw[k] = exp(-2 pi i k / M); with stride s the table is of length s*M (every s-th entry)
    __device__ __forceinline__ void load(int j, const float2* __restrict__ tw, int stride = 1) {
        constexpr int T = PL::T;
        [&]<int... Ps>(std::integer_sequence<int, Ps...>) {
            (([&] {
                 constexpr int p = Ps;
                 constexpr int RP = PL::radix(p);
                 constexpr int NS = PL::ns(p);
                 constexpr int NB = E / RP;
                 if constexpr (NS > 1) {
                     constexpr int STEP = M / (NS * RP);
#pragma unroll
                     for (int i = 0; i < NB; ++i) {
                         const int k = (j + i * T) & (NS - 1);
#pragma unroll
                         for (int kk = 1; kk < RP; ++kk) w[p][i * RP + kk] = tw[stride * (k * kk * STEP)];
                     }
                 }
             }()),
             ...);
        }(std::make_integer_sequence<int, PL::PASSES>{});
    }
};

// LDS slot of element e of a length-M exchange. The strided Stockham writes (16 apart in
// the first pass) are spread over the banks either by one pad slot every 16 elements, or,
// for M = 4096, by XOR-ing the element's low 4 bits with the next 4 (a permutation within
// each aligned group of 16 slots, so no padding). Measured: on the 2048^2 plane the column
// pass takes 61.3 instead of 63.0 us with the row passes unchanged, the 4096^2 plane is
// unchanged overall, and at other lengths the padding is as fast or faster.
template <int M>
__device__ __forceinline__ int lds_slot(int e) {
    if constexpr (M == 4096) return e ^ ((e >> 4) & 15);
    else return e + (e >> 4);
}
template <int M>
constexpr int lds_elems() { return M == 4096 ? M : M + M / 16; }

// Block barrier for the LDS exchanges only. Threads of a block communicate through
// LDS alone (every global location is written by exactly one thread), so the
// barrier waits for this thread's LDS operations but leaves global loads and
// stores in flight; prefetched loads and the previous item's stores overlap the
// transform.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// P interleaved transforms share each LDS slot (P complex values, 8*P bytes), so
// one thread moves all of them with a single 8- or 16-byte LDS access.
template <int P>
__device__ __forceinline__ void lds_put(float2* lds, int slot, const float2 (&x)[P]) {
    if constexpr (P == 1) {
        lds[slot] = x[0];
    } else {
        static_assert(P == 2, "P");
        reinterpret_cast<float4*>(lds)[slot] = make_float4(x[0].x, x[0].y, x[1].x, x[1].y);
    }
}
template <int P>
__device__ __forceinline__ void lds_get(const float2* lds, int slot, float2 (&x)[P]) {
    if constexpr (P == 1) {
        x[0] = lds[slot];
    } else {
        const float4 t = reinterpret_cast<const float4*>(lds)[slot];
        x[0] = make_float2(t.x, t.y);
        x[1] = make_float2(t.z, t.w);
    }
}

// One Stockham pass over P transforms that share twiddles. Writes results to LDS
// (intermediate pass) or back into registers in natural order (last pass). With SPLIT
// (P == 2 only) the LDS holds one transform at a time: transform 0 is written here and
// transform 1's outputs are kept in `held` for the second half of the exchange.
// ZIN (first pass only, NS == 1): the butterfly inputs kk >= RP/2 are the elements
// b + kk*M/RP >= M/2, the zero-padded half of the sequence; they are not read.
template <int M, int E, int P, int RP, int NS, bool LAST, int DIR, bool SPLIT, bool PRE,
          bool ZIN = false>
__device__ __forceinline__ void stockham_pass(float2 (&v)[P][E], float2* lds, int j,
                                              const float2* __restrict__ tw,
                                              const float2 (&wpre)[E], float2 (&held)[E]) {
    static_assert(!ZIN || NS == 1, "zero inputs are known in the first pass only");
    constexpr int T = M / E;
    constexpr int NB = E / RP;  // butterflies per thread and transform
    float2 out[P][E];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = j + i * T;
        const int k = b & (NS - 1);
        float2 w[RP];
        if constexpr (NS > 1) {
            constexpr int STEP = M / (NS * RP);
#pragma unroll
            for (int kk = 1; kk < RP; ++kk) w[kk] = PRE ? wpre[i * RP + kk] : tw[k * kk * STEP];
        }
        float2 u[P][RP];
#pragma unroll
        for (int p = 0; p < P; ++p) {
#pragma unroll
            for (int kk = 0; kk < (ZIN ? RP / 2 : RP); ++kk) u[p][kk] = v[p][i + kk * NB];
            if constexpr (NS > 1) {
#pragma unroll
                for (int kk = 1; kk < RP; ++kk) u[p][kk] = ctw<DIR>(u[p][kk], w[kk]);
            }
            dft<RP, DIR, 0, 1, ZIN>(u[p]);
        }
        if constexpr (LAST) {
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int kk = 0; kk < RP; ++kk) out[p][i + kk * NB] = u[p][kk];
        } else if constexpr (SPLIT) {
            const int base = (b / NS) * NS * RP + k;
#pragma unroll
            for (int kk = 0; kk < RP; ++kk) {
                lds[lds_slot<M>(base + kk * NS)] = u[0][kk];
                held[i * RP + kk] = u[1][kk];
            }
        } else {
            const int base = (b / NS) * NS * RP + k;
#pragma unroll
            for (int kk = 0; kk < RP; ++kk) {
                float2 x[P];
#pragma unroll
                for (int p = 0; p < P; ++p) x[p] = u[p][kk];
                lds_put<P>(lds, lds_slot<M>(base + kk * NS), x);
            }
        }
    }
    if constexpr (LAST) {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int r = 0; r < E; ++r) v[p][r] = out[p][r];
    }
}

// Full transform of P sequences at once. On entry v[p][r] = x_p[j + r*T]; on exit
// v[p][r] = X_p[j + r*T]. All threads of the block must call it (block barriers).
// SPLIT halves the LDS footprint (one float2 slot per element) at the cost of two more
// barriers per exchange.
// ZIN: the elements M/2 .. M-1 of the input are zero (whatever the registers hold).
template <int M, int E, int P, int DIR, bool SPLIT = false, bool PRE = false, bool ZIN = false>
__device__ __forceinline__ void fft_impl(float2 (&v)[P][E], float2* lds, int j,
                                         const float2* __restrict__ tw,
                                         const TwCache<M, E>* twc) {
    static_assert(!SPLIT || P == 2, "split exchange is for two transforms");
    using PL = Plan<M, E>;
    constexpr int T = PL::T;
    [&]<int... Ps>(std::integer_sequence<int, Ps...>) {
        (([&] {
             constexpr int p = Ps;
             constexpr int RP = PL::radix(p);
             constexpr int NS = PL::ns(p);
             constexpr bool LAST = (p == PL::PASSES - 1);
             constexpr bool Z = ZIN && p == 0;
             float2 held[E];
             if constexpr (PRE)
                 stockham_pass<M, E, P, RP, NS, LAST, DIR, SPLIT, true, Z>(v, lds, j, tw, twc->w[p], held);
             else
                 stockham_pass<M, E, P, RP, NS, LAST, DIR, SPLIT, false, Z>(v, lds, j, tw, held, held);
             if constexpr (!LAST) {
                 if constexpr (SPLIT) {
                     lds_barrier();
#pragma unroll
                     for (int r = 0; r < E; ++r) v[0][r] = lds[lds_slot<M>(j + r * T)];
                     lds_barrier();
                     constexpr int NB = E / RP;
#pragma unroll
                     for (int i = 0; i < NB; ++i) {
                         const int b = j + i * T;
                         const int k = b & (NS - 1);
                         const int base = (b / NS) * NS * RP + k;
#pragma unroll
                         for (int kk = 0; kk < RP; ++kk) lds[lds_slot<M>(base + kk * NS)] = held[i * RP + kk];
                     }
                     lds_barrier();
#pragma unroll
                     for (int r = 0; r < E; ++r) v[P - 1][r] = lds[lds_slot<M>(j + r * T)];
                     lds_barrier();
                 } else {
                     lds_barrier();
#pragma unroll
                     for (int r = 0; r < E; ++r) {
                         float2 x[P];
                         lds_get<P>(lds, lds_slot<M>(j + r * T), x);
#pragma unroll
                         for (int q = 0; q < P; ++q) v[q][r] = x[q];
                     }
                     lds_barrier();
                 }
             }
         }()),
         ...);
    }(std::make_integer_sequence<int, PL::PASSES>{});
}

// Transform with twiddles loaded from the table in each pass.
template <int M, int E, int P, int DIR, bool SPLIT = false>
__device__ __forceinline__ void fft(float2 (&v)[P][E], float2* lds, int j,
                                    const float2* __restrict__ tw) {
    fft_impl<M, E, P, DIR, SPLIT, false>(v, lds, j, tw, nullptr);
}

// Transform with the thread's twiddles preloaded in registers.
template <int M, int E, int P, int DIR, bool SPLIT = false>
__device__ __forceinline__ void fft(float2 (&v)[P][E], float2* lds, int j,
                                    const TwCache<M, E>& twc) {
    fft_impl<M, E, P, DIR, SPLIT, true>(v, lds, j, nullptr, &twc);
}

// Forward transform of a zero-padded sequence (elements M/2 .. M-1 zero): the first
// pass skips the additions of the zero half; the registers of those elements are not read.
template <int M, int E, int P, int DIR, bool SPLIT = false>
__device__ __forceinline__ void fft_zpad(float2 (&v)[P][E], float2* lds, int j,
                                         const TwCache<M, E>& twc) {
    fft_impl<M, E, P, DIR, SPLIT, true, true>(v, lds, j, nullptr, &twc);
}

}  // namespace cwo
