// Column pass of the shifted angular spectrum method (Sec. 2.1.5, Eqs. shift_ang1 and
// shift_ang2): the angular-spectrum transfer function times the linear phase
// exp(i 2 pi (ox fx + oy fy)), which moves the destination window by (ox, oy), and times
// the band-limit functions Rect((fx - cx)/wx) Rect((fy - cy)/wy). The extra factors
// separate into one term per column and one per row: folded into the phase terms of the
// fast phase form, or as complex factors on top of the exact form.

#include "column.hpp"

namespace cwo {

// Band-limit masks, one 0/1 value per column and per row, computed once per call:
// Rect((f - c)/w) for f = signed bin index * df, the test (f - c)/w in [-1/2, 1/2]
// evaluated in FP64 with each operation rounded on its own (an integer decision from
// floating point: the same operations as an FP64 evaluation of the definition); w <= 0
// means no limit. tab = [x masks (mx) | y masks (my)].
__global__ void k_band_masks(float* __restrict__ tab, int mx, int my, double dfx, double dfy,
                             AsmShift sh) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= mx + my) return;
    const bool xa = i < mx;
    const int p = xa ? i : i - mx, m = xa ? mx : my;
    const double c = xa ? sh.cx : sh.cy, w = xa ? sh.wx : sh.wy;
    float v = 1.0f;
    if (w > 0.0) {
        const double f = (double)(p < m / 2 ? p : p - m) * (xa ? dfx : dfy);
        const double t = (f - c) / w;
        v = (fabs(t) <= 0.5) ? 1.0f : 0.0f;
    }
    tab[i] = v;
}

// offset * f in revolutions, f = signed bin index * df (FP64)
__device__ __forceinline__ double shift_rev(int p, int m, double df, double offset) {
    return offset * ((double)(p < m / 2 ? p : p - m) * df);
}

// Any base form: one complex factor per column and per row, exp(i 2 pi offset f) times
// the band mask, the phase reduced modulo one revolution in FP64 before the FP32 sine and
// cosine (which take revolutions).
__device__ __forceinline__ float2 shift_factor(int p, int m, double df, double offset, float mk) {
    const double u = shift_rev(p, m, df, offset);
    const float r = (float)(u - rint(u));
    return make_float2(mk * __builtin_amdgcn_cosf(r), mk * __builtin_amdgcn_sinf(r));
}

template <class Base>
struct ShiftedH {
    Base b;
    double dfx, dfy;
    AsmShift sh;
    const float* __restrict__ mask;  // [mx | my] band masks
    int mx, my;
    struct Col {
        typename Base::Col c;
        float2 e;
    };
    struct Row {
        typename Base::Row r;
        float2 e;
    };
    __device__ __forceinline__ Col column(int p) const {
        return Col{b.column(p), shift_factor(p, mx, dfx, sh.ox, mask[p])};
    }
    __device__ __forceinline__ Row row(int q) const {
        return Row{b.row(q), shift_factor(q, my, dfy, sh.oy, mask[mx + q])};
    }
    __device__ __forceinline__ float2 operator()(const Col& c, const Row& r) const {
        return cmul(b(c.c, r.r), cmul(c.e, r.e));
    }
};

// Fast phase form with the shift folded into its phase terms: the column term gains
// +reduced(ox fx) and the row term -oy fy (FP64, reduced together with the rest of the
// row phase), so no extra sine or cosine is taken; the band limits are 0/1 factors.
struct ShiftedFast {
    AsmHFast b;
    double dfx, dfy;
    AsmShift sh;
    const float* __restrict__ mask;  // [mx | my] band masks
    int mx, my;
    struct Col {
        AsmHFast::Col c;
        float m;
    };
    struct Row {
        AsmHFast::Row r;
        float m;
    };
    __device__ __forceinline__ Col column(int p) const {
        Col k{b.column(p), mask[p]};
        const double t = shift_rev(p, mx, dfx, sh.ox);
        k.c.ca += (float)(t - rint(t));  // stays within [-1.5, 1.5]; reduced once more per bin
        return k;
    }
    __device__ __forceinline__ Row row(int q) const {
        Row k{b.row(q), mask[mx + q]};
        k.r.hb -= shift_rev(q, my, dfy, sh.oy);
        return k;
    }
    __device__ __forceinline__ float2 operator()(const Col& c, const Row& r) const {
        const float2 h = b(c.c, r.r);
        const float m = c.m * r.m;
        return make_float2(h.x * m, h.y * m);
    }
};

template <class HF, class ST>
static hipError_t launch_shifted_t(void* buf, int ny, int my, int mx, const HF& hf, float hscale,
                                   const float2* tw, hipStream_t s, int layout) {
    using SE = typename ST::E;
    const bool half = (my == 2 * ny);
    if (layout == 1 && (!half || mx % kTileW != 0)) return hipErrorInvalidValue;
    CWO_DISPATCH_M(my, {
        using C = ColCfg<MM>;
        const int items = (mx + C::COLS - 1) / C::COLS;
        if (half && layout == 1) {
            if constexpr (MM == 8192)  // two transforms of 4096 per column, one per block
                launch_kernel((k_col_split<MM / 2, HF, ST, LayTile>), dim3(mx), dim3(MM / 32),
                                   0, s, (SE*)buf, ny, mx, 1, (size_t)0, hf, hscale, tw,
                                   LayTile{ny});
            else
                launch_kernel((k_col<MM, true, HF, ST, LayTile>), dim3(items),
                                   dim3(C::THREADS), 0, s, (SE*)buf, ny, mx, 1, (size_t)0, hf,
                                   hscale, tw, LayTile{ny});
        } else if (half) {
            launch_kernel((k_col<MM, true, HF, ST, LayRow>), dim3(items), dim3(C::THREADS),
                               0, s, (SE*)buf, ny, mx, 1, (size_t)0, hf, hscale, tw, LayRow{mx});
        } else if constexpr (std::is_same_v<ST, StF32>) {
            launch_kernel((k_col<MM, false, HF, ST, LayRow>), dim3(items), dim3(C::THREADS),
                               0, s, (SE*)buf, ny, mx, 1, (size_t)0, hf, hscale, tw, LayRow{mx});
        } else {
            return hipErrorInvalidValue;
        }
    });
    return hipGetLastError();
}

template <class HF>
static hipError_t launch_shifted_prec(void* buf, int ny, int my, int mx, const HF& hf,
                                      const Storage& st, const float2* tw, hipStream_t s) {
    switch (st.prec) {
        case 0: return launch_shifted_t<HF, StF32>(buf, ny, my, mx, hf, st.col_scale, tw, s, st.layout);
        case 1: return launch_shifted_t<HF, StF16>(buf, ny, my, mx, hf, st.col_scale, tw, s, st.layout);
        case 2: return launch_shifted_t<HF, StBF16>(buf, ny, my, mx, hf, st.col_scale, tw, s, st.layout);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_col_asm_shifted(void* buf, int ny, int my, int mx, const AsmScalars& a,
                                  const AsmShift& sh, float* masks, const Storage& st,
                                  const float2* tw, hipStream_t s) {
    launch_kernel(k_band_masks, dim3((mx + my + 255) / 256), dim3(256), 0, s, masks, mx, my,
                       a.dfx, a.dfy, sh);
    const double sx = a.lam * (0.5 * mx) * a.dfx, sy = a.lam * (0.5 * my) * a.dfy;
    if (sx * sx + sy * sy <= kAsmFastMaxS) {
        ShiftedFast hf;
        hf.b.lam_dfx = a.lam * a.dfx;
        hf.b.lam_dfy = a.lam * a.dfy;
        hf.b.zl = a.zl;
        hf.b.half_zl = 0.5 * a.zl;
        hf.b.c0 = (float)(a.zl - std::nearbyint(a.zl));
        hf.b.mx = mx;
        hf.b.my = my;
        hf.dfx = a.dfx;
        hf.dfy = a.dfy;
        hf.sh = sh;
        hf.mask = masks;
        hf.mx = mx;
        hf.my = my;
        return launch_shifted_prec(buf, ny, my, mx, hf, st, tw, s);
    }
    ShiftedH<AsmH> hf{AsmH{a.dfx, a.dfy, a.lam, a.zl, mx, my}, a.dfx, a.dfy, sh, masks, mx, my};
    return launch_shifted_prec(buf, ny, my, mx, hf, st, tw, s);
}

}  // namespace cwo
