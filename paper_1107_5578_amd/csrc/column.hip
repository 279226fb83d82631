// Host launchers of the column pass (forward FFT along y, transfer function, inverse FFT,
// crop) for the plain, batched and mixed-batch forms; the kernel is in column.hpp.

#include "column.hpp"

namespace cwo {

// On the tiled plane a padded column of 8192 runs by default as two transforms of 4096 (one
// column per block), shorter ones as one transform per column (two columns per thread).
// ALT launchers (single planes, where the autotuner may pick the column form) also build the
// other form at 4096 and 8192: col_form 1 full length, 2 split.
template <class HF, class ST, bool ALT = false>
static hipError_t launch_col_t(void* buf, int ny, int my, int mx, int batch, size_t plane,
                               const HF& hf, float hscale, const float2* tw, hipStream_t s,
                               int layout = 0, int col_form = 0) {
    const bool half = (my == 2 * ny);
    using SE = typename ST::E;
    if (layout == 1 && (!half || mx % kTileW != 0)) return hipErrorInvalidValue;
    CWO_DISPATCH_M(my, {
        using C = ColCfg<MM>;
        const int items = (mx + C::COLS - 1) / C::COLS * batch;
        if (half && layout == 1) {
            constexpr bool CAN_SPLIT = MM == 8192 || (ALT && MM == 4096);
            constexpr bool CAN_FULL = MM != 8192 || ALT;
            const bool split = MM == 8192 ? col_form != 1 : col_form == 2;
            if (split) {
                if constexpr (CAN_SPLIT)
                    launch_kernel((k_col_split<MM / 2, HF, ST, LayTile>), dim3(mx * batch),
                                       dim3(MM / 32), 0, s, (SE*)buf, ny, mx, batch, plane, hf,
                                       hscale, tw, LayTile{ny});
                else
                    return hipErrorInvalidValue;
            } else {
                if constexpr (CAN_FULL)
                    launch_kernel((k_col<MM, true, HF, ST, LayTile>), dim3(items),
                                       dim3(C::THREADS), 0, s, (SE*)buf, ny, mx, batch, plane, hf,
                                       hscale, tw, LayTile{ny});
                else
                    return hipErrorInvalidValue;
            }
        } else if (half) {
            launch_kernel((k_col<MM, true, HF, ST, LayRow>), dim3(items), dim3(C::THREADS), 0,
                               s, (SE*)buf, ny, mx, batch, plane, hf, hscale, tw, LayRow{mx});
        } else if constexpr (std::is_same_v<ST, StF32>) {
            launch_kernel((k_col<MM, false, HF, ST, LayRow>), dim3(items), dim3(C::THREADS),
                               0, s, (SE*)buf, ny, mx, batch, plane, hf, hscale, tw, LayRow{mx});
        } else {
            return hipErrorInvalidValue;
        }
    });
    return hipGetLastError();
}

template <class HF>
static hipError_t launch_col_impl(void* buf, int ny, int my, int mx, int batch, size_t plane,
                                  const HF& hf, const Storage& st, const float2* tw,
                                  hipStream_t s) {
    switch (st.prec) {
        case 0: return launch_col_t<HF, StF32, true>(buf, ny, my, mx, batch, plane, hf, st.col_scale, tw, s, st.layout, st.col_form);
        case 1: return launch_col_t<HF, StF16, true>(buf, ny, my, mx, batch, plane, hf, st.col_scale, tw, s, st.layout, st.col_form);
        case 2: return launch_col_t<HF, StBF16, true>(buf, ny, my, mx, batch, plane, hf, st.col_scale, tw, s, st.layout, st.col_form);
    }
    return hipErrorInvalidValue;
}

PlaneTF asm_plane_tf(const AsmScalars& a, int mx, int my) {
    PlaneTF r{};
    // largest s = (lambda fx)^2 + (lambda fy)^2 on the grid: the Nyquist corner
    const double sx = a.lam * (0.5 * mx) * a.dfx, sy = a.lam * (0.5 * my) * a.dfy;
    const double smax = sx * sx + sy * sy;
    if (smax <= kAsmFastMaxS) {
        // the series to s^4 suffices when |zl| times its remainder, at most
        // c_5 smax^5/(1 - smax) with c_5 = 7/256, stays below 2^-28 revolution
        const double s5 = smax * smax * smax * smax * smax;
        r.form = std::fabs(a.zl) * (7.0 / 256.0) * s5 / (1.0 - smax) <= std::ldexp(1.0, -28) ? 0 : 1;
        r.d0 = a.lam * a.dfx;
        r.d1 = a.lam * a.dfy;
        r.d2 = a.zl;
        r.d3 = 0.5 * a.zl;
        r.c0 = (float)(a.zl - std::nearbyint(a.zl));
    } else {
        r.form = 2;
        r.d0 = a.dfx;
        r.d1 = a.dfy;
        r.d2 = a.lam;
        r.d3 = a.zl;
    }
    return r;
}

hipError_t launch_col_asm(void* buf, int ny, int my, int mx, int batch, size_t plane,
                          const AsmScalars& a, const Storage& st, const float2* tw, hipStream_t s) {
    const PlaneTF r = asm_plane_tf(a, mx, my);
    if (r.form <= 1) {
        auto fill = [&](auto& hf) {
            hf.lam_dfx = r.d0;
            hf.lam_dfy = r.d1;
            hf.zl = r.d2;
            hf.half_zl = r.d3;
            hf.c0 = r.c0;
            hf.mx = mx;
            hf.my = my;
        };
        if (r.form == 0) {
            AsmHFastN<4> hf;
            fill(hf);
            return launch_col_impl(buf, ny, my, mx, batch, plane, hf, st, tw, s);
        }
        AsmHFastN<9> hf;
        fill(hf);
        return launch_col_impl(buf, ny, my, mx, batch, plane, hf, st, tw, s);
    }
    AsmH hf{a.dfx, a.dfy, a.lam, a.zl, mx, my};
    return launch_col_impl(buf, ny, my, mx, batch, plane, hf, st, tw, s);
}

hipError_t launch_col_mixed(float2* buf, int ny, int my, int mx, int n, size_t plane,
                            const PlaneTF* tf, int form, const float2* tw, hipStream_t s,
                            int layout) {
    // complex64 only (mixed batches are not built for 16-bit storage)
    if (form == 0 || form == 1) {
        auto run = [&](auto& list) {
            for (int k = 0; k < n; ++k) {
                if (tf[k].form != form) continue;
                auto& f = list.f[list.n];
                f.lam_dfx = tf[k].d0;
                f.lam_dfy = tf[k].d1;
                f.zl = tf[k].d2;
                f.half_zl = tf[k].d3;
                f.c0 = tf[k].c0;
                f.mx = mx;
                f.my = my;
                list.idx[list.n++] = k;
            }
            return list.n ? launch_col_t<std::decay_t<decltype(list)>, StF32>(
                                (void*)buf, ny, my, mx, list.n, plane, list, 1.0f, tw, s, layout)
                          : hipSuccess;
        };
        if (form == 0) {
            PlaneList<AsmHFastN<4>> l{};
            return run(l);
        }
        PlaneList<AsmHFastN<9>> l{};
        return run(l);
    }
    if (form == 3) {
        PlaneList<FresnelH> l{};
        for (int k = 0; k < n; ++k) {
            if (tf[k].form != 3) continue;
            l.f[l.n] = FresnelH{tf[k].h, tf[k].h + mx};
            l.idx[l.n++] = k;
        }
        return l.n ? launch_col_t<PlaneList<FresnelH>, StF32>((void*)buf, ny, my, mx, l.n, plane, l,
                                                               1.0f, tw, s, layout)
                   : hipSuccess;
    }
    return hipErrorInvalidValue;  // the exact ASM form is not batched
}

hipError_t launch_col_asm(float2* buf, int ny, int my, int mx, int batch, size_t plane,
                          const AsmScalars& a, const float2* tw, hipStream_t s, int layout) {
    Storage st;
    st.layout = layout;
    return launch_col_asm((void*)buf, ny, my, mx, batch, plane, a, st, tw, s);
}

hipError_t launch_col_fresnel(void* buf, int ny, int my, int mx, int batch, size_t plane,
                              const float2* hx, const float2* hy, const Storage& st,
                              const float2* tw, hipStream_t s) {
    FresnelH hf{hx, hy};
    return launch_col_impl(buf, ny, my, mx, batch, plane, hf, st, tw, s);
}

}  // namespace cwo
