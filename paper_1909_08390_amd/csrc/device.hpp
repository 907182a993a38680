// Device helpers shared by the forward and adjoint kernels (not part of
// the ABI): table access through the constant address space, ghost-node
// addressing, the one-axis equilibrium factor and the MP-9 face rule.
#pragma once

#include "common.hpp"

namespace imexlb {
namespace {

// Tables are read through the constant address space so that uniform
// accesses become scalar loads.
#define IMEXLB_CONST __attribute__((address_space(4)))
// Lambdas of the kernel bodies are inlined even where they are called twice.
#define IMEXLB_INLINE __attribute__((always_inline))
typedef const DevTables IMEXLB_CONST CTab;
typedef const double IMEXLB_CONST* CDp;


// Ghost-node addressing (Sec. IV): outflow copies the boundary node,
// periodic wraps.
__device__ __forceinline__ int bc_map(int i, int n, int bc) {
    if (bc == 1) {
        i %= n;
        return i < 0 ? i + n : i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// One-axis factor of the discrete equilibrium, Eq. (gExpanded):
// g_k = w_k sum_l He_l(p_k)/l! a_l with a_l = sum_s l!/(2^s s!(l-2s)!) (T-1)^s u^(l-2s).
// The a_l satisfy a_0 = 1, a_1 = u, a_{l+1} = u a_l + l (T-1) a_{l-1}
// (they are E[He_l(X)] for X ~ N(u, T)); h[l] = w_k He_l(p_k)/l! is tabulated.
__device__ __forceinline__ double herm_factor(CDp h, int Q, double u,
                                              double th) {
    double am = 1.0, ac = u;
    double g = fma(h[1], u, h[0]);
    double lth = th;  // l (T - 1)
    for (int l = 1; l < Q - 1; ++l) {
        const double an = fma(u, ac, lth * am);
        g = fma(h[l + 1], an, g);
        am = ac;
        ac = an;
        lth += th;
    }
    return g;
}

// Median, three-way min / max.  FP32 has single instructions for them
// (v_med3_f32, v_min3_f32, v_max3_f32); FP64 composes two-way min / max.
template <typename R>
__device__ __forceinline__ R med3(R a, R b, R c) {
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_fmed3f(a, b, c);
    else return fmax(fmin(a, b), fmin(fmax(a, b), c));
}

template <typename R>
__device__ __forceinline__ R min3(R a, R b, R c) {
    return fmin(fmin(a, b), c);
}

template <typename R>
__device__ __forceinline__ R max3(R a, R b, R c) {
    return fmax(fmax(a, b), c);
}

// x clipped to [lo, hi] (lo <= hi).
template <typename R>
__device__ __forceinline__ R clamp(R x, R lo, R hi) {
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_fmed3f(x, lo, hi);
    else return fmin(fmax(x, lo), hi);
}

// Two-argument minmod: the signed smaller magnitude when both share a sign,
// else 0; equal to the median of (0, a, b), i.e. 0 clamped to
// [min(a, b), max(a, b)].
template <typename R>
__device__ __forceinline__ R minmod2(R a, R b) {
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_fmed3f(R(0), a, b);
    else return fmin(fmax(fmin(a, b), R(0)), fmax(a, b));
}

// Four-argument minmod: signed smallest magnitude when all share a sign,
// else 0; equal to 0 clamped to [min, max] of the four arguments.
template <typename R>
__device__ __forceinline__ R minmod4(R a, R b, R c, R d) {
    const R mn = min3(a, b, fmin(c, d));
    const R mx = max3(a, b, fmax(c, d));
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_fmed3f(R(0), mn, mx);
    else return fmin(fmax(mn, R(0)), mx);
}

// MP-9 interface value (Sec. IV) of the face between F_s and F_{s+1} for
// flow towards +s, from the first differences dd[k] = F_{s-3+k} - F_{s-4+k}
// (k = 0 .. 7) of the nine upwind-biased nodes.
//
// F^L is evaluated in difference form: 2520 (F^L - F_s) = sum_k c_k dd[k]
// with c = (-4, 37, -162, 479, 1120, -255, 50, -5), the paper's nine weights
// (times 2520) re-expressed on first differences, so uniform data give
// F^L = F_s exactly and every weight is a small integer.  F^MP = median(F_s,
// F_{s+1}, F^UL) with F^UL = F_s + 4 (F_s - F_{s-1}) equals F_s + minmod(
// F_{s+1} - F_s, 4 (F_s - F_{s-1})), so the monotonicity test
// (F^L - F_s)(F^L - F^MP) <= 0 needs no median.  When it fails the face is
// F^L clipped to [F^min, F^max] built from the M4 curvatures.  The clipping
// work is kept inside its branch (the caller passes opaque copies of its
// inputs, so the compiler cannot hoist it), and a wavefront none of whose
// lanes needs it skips it.
template <typename R>
__device__ __forceinline__ void opaque(R& x) {
    asm volatile("" : "+v"(x));
}

// Linear part and monotonicity test of one face: returns F^L and sets q,
// positive when the face must be clipped (q = (F^L - F_s)(F^L - F^MP)
// times 2520), and t = 4 (F_s - F_{s-1}) = F^UL - F_s.
template <typename R>
__device__ __forceinline__ R mp9_face_linear(const R (&dd)[8], R fs, R& t, R& q) {
    R s = R(-4) * dd[0];
    s = fma(R(37), dd[1], s);
    s = fma(R(-162), dd[2], s);
    s = fma(R(479), dd[3], s);
    s = fma(R(1120), dd[4], s);
    s = fma(R(-255), dd[5], s);
    s = fma(R(50), dd[6], s);
    s = fma(R(-5), dd[7], s);
    constexpr R inv = R(1.0 / 2520.0);
    t = R(4) * dd[3];
    const R mm = minmod2(dd[4], t);  // F^MP - F_s
    q = s * fma(s, inv, -mm);
    return fma(s, inv, fs);
}

// M4 limit between two curvatures: minmod4(4 a - b, 4 b - a, a, b), the
// d^M4 of the F^LC and F^MD bounds (a = C_{s-1}, b = C_s gives the limit at
// s - 1/2; a = C_s, b = C_{s+1} the one at s + 1/2).
template <typename R>
__device__ __forceinline__ R mp9_m4(R a, R b) {
    return minmod4(fma(R(4), a, -b), fma(R(4), b, -a), a, b);
}

// F^L limited to [F^min, F^max] from the face's nodes F_s, F_{s+1}, t =
// F^UL - F_s, the differences dm1 = F_s - F_{s-1} and d0 = F_{s+1} - F_s,
// and the M4 limits at s - 1/2 (mlo) and s + 1/2 (mhi).
template <typename R>
__device__ __forceinline__ R mp9_face_bound(R f, R g, R u, R dm1, R d0, R mlo, R mhi, R fl) {
    const R ul = f + u;
    const R lc = fma(R(4.0 / 3.0), mlo, fma(R(0.5), dm1, f));
    const R md = fma(R(0.5), d0 - mhi, f);
    R lo, hi;  // F^min <= F_s <= F^max
    if constexpr (sizeof(R) == 4) {
        lo = fmax(min3(f, g, md), min3(f, ul, lc));
        hi = fmin(max3(f, g, md), max3(f, ul, lc));
    } else {
        // without three-way FP64 min / max: max(min(F_s, A, B), min(F_s, C, D))
        // = min(F_s, max(min(A, B), min(C, D))), min(F_s, .) being monotone
        // (exact; four operations instead of five), and F^max likewise
        lo = fmin(f, fmax(fmin(g, md), fmin(ul, lc)));
        hi = fmax(f, fmin(fmax(g, md), fmax(ul, lc)));
    }
    return clamp(fl, lo, hi);
}


}  // namespace
}  // namespace imexlb
