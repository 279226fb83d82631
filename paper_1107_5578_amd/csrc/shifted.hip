// Column pass of the shifted angular spectrum method (Sec. 2.1.5, Eqs. shift_ang1 and
// shift_ang2): the angular-spectrum transfer function times the linear phase
// exp(i 2 pi (ox fx + oy fy)), which moves the destination window by (ox, oy), and times
// the band-limit functions Rect((fx - cx)/wx) Rect((fy - cy)/wy). The extra factors
// separate into one complex number per column and one per row.

#include "column.hpp"

namespace cwo {

// exp(i 2 pi offset f) * Rect((f - c)/w) for f = signed bin index * df. The bin test
// (f - c)/w in [-1/2, 1/2] and the phase are evaluated in FP64 without contraction (an
// integer decision from floating point: the same operations as an FP64 evaluation of
// the definition); the phase is reduced modulo one revolution before the FP32 sine and
// cosine, which take revolutions.
__device__ __forceinline__ float2 shift_factor(int p, int m, double df, double offset, double c,
                                               double w) {
#pragma clang fp contract(off)
    const double f = (double)(p < m / 2 ? p : p - m) * df;
    if (w > 0.0) {
        const double t = (f - c) / w;
        if (!(fabs(t) <= 0.5)) return make_float2(0.f, 0.f);
    }
    const double u = offset * f;
    const float r = (float)(u - rint(u));
    return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
}

template <class Base>
struct ShiftedH {
    Base b;
    double dfx, dfy;
    AsmShift sh;
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
        return Col{b.column(p), shift_factor(p, mx, dfx, sh.ox, sh.cx, sh.wx)};
    }
    __device__ __forceinline__ Row row(int q) const {
        return Row{b.row(q), shift_factor(q, my, dfy, sh.oy, sh.cy, sh.wy)};
    }
    __device__ __forceinline__ float2 operator()(const Col& c, const Row& r) const {
        return cmul(b(c.c, r.r), cmul(c.e, r.e));
    }
};

template <class HF>
static hipError_t launch_shifted_t(float2* buf, int ny, int my, int mx, const HF& hf,
                                   const float2* tw, hipStream_t s) {
    const bool half = (my == 2 * ny);
    CWO_DISPATCH_M(my, {
        using C = ColCfg<MM>;
        const int items = (mx + C::COLS - 1) / C::COLS;
        if (half)
            hipLaunchKernelGGL((k_col<MM, true, HF, StF32>), dim3(items), dim3(C::THREADS), 0, s,
                               buf, ny, mx, 1, (size_t)0, hf, 1.0f, tw);
        else
            hipLaunchKernelGGL((k_col<MM, false, HF, StF32>), dim3(items), dim3(C::THREADS), 0, s,
                               buf, ny, mx, 1, (size_t)0, hf, 1.0f, tw);
    });
    return hipGetLastError();
}

hipError_t launch_col_asm_shifted(float2* buf, int ny, int my, int mx, const AsmScalars& a,
                                  const AsmShift& sh, const float2* tw, hipStream_t s) {
    const double sx = a.lam * (0.5 * mx) * a.dfx, sy = a.lam * (0.5 * my) * a.dfy;
    if (sx * sx + sy * sy <= kAsmFastMaxS) {
        ShiftedH<AsmHFast> hf;
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
        hf.mx = mx;
        hf.my = my;
        return launch_shifted_t(buf, ny, my, mx, hf, tw, s);
    }
    ShiftedH<AsmH> hf{AsmH{a.dfx, a.dfy, a.lam, a.zl, mx, my}, a.dfx, a.dfy, sh, mx, my};
    return launch_shifted_t(buf, ny, my, mx, hf, tw, s);
}

}  // namespace cwo
