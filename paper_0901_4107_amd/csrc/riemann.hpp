// riemann.hpp -- exact Riemann solver for the 1D Euler equations of an ideal
// gas, sampled at x/t = 0, for one face per lane (Section 3.3: the flux
// uses an exact solver extended to vacuum states). Templated on the working
// precision so the same wave logic serves the double and the single path.
//
// The star pressure is the root of f(p) = f_L(p) + f_R(p) + (u_R - u_L),
// where each side contributes the Rankine-Hugoniot branch (p > p_K) or the
// isentropic branch (p <= p_K). f is increasing and concave, so Newton's
// method from any positive start lands at or below the root after one step
// and then rises monotonically to it; a step that lands at p <= 0 is
// replaced by a tenth of the previous iterate.
//
// Cost notes (gfx950): powers are exp2(y log2 x) with the hardware v_exp/v_log
// in float, and exp(y ln x) from short series in double (mm_pow below; a
// few ulp, far below the parity bound). u* and the star-state
// powers reuse the last Newton evaluation with a first-order correction in
// the final step (error O(step^2), below 1e-18 relative at convergence), and
// integer exponents 2/(g-1) (3 for g = 5/3, 5 for g = 7/5) are multiplied out.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace mm {

enum RiemannCase : int { RC_NORMAL = 0, RC_LEFT_VACUUM = 1, RC_RIGHT_VACUUM = 2,
                         RC_VACUUM_GENERATED = 3, RC_BOTH_VACUUM = 4 };

// Constants of the equation of state, built once on the host.
template <typename T> struct GasConst {
    T g, z, inv_z, zs1, zs2, gm_ratio, two_over_gm1, two_over_gp1, gm1_over_2, g_over_gm1, exp_rho;
    int iexp_rho;   // 2/(g-1) when it is a small integer, else 0
    __host__ __device__ GasConst() {}
    __host__ explicit GasConst(double gamma) {
        g = (T)gamma;
        z = (T)((gamma - 1.0) / (2.0 * gamma));
        inv_z = (T)(2.0 * gamma / (gamma - 1.0));
        zs1 = (T)((gamma + 1.0) / (2.0 * gamma));
        zs2 = (T)((gamma - 1.0) / (2.0 * gamma));
        gm_ratio = (T)((gamma - 1.0) / (gamma + 1.0));
        two_over_gm1 = (T)(2.0 / (gamma - 1.0));
        two_over_gp1 = (T)(2.0 / (gamma + 1.0));
        gm1_over_2 = (T)(0.5 * (gamma - 1.0));
        g_over_gm1 = (T)(gamma / (gamma - 1.0));
        const double e = 2.0 / (gamma - 1.0);
        exp_rho = (T)e;
        const double r = (double)(long)(e + 0.5);
        iexp_rho = (r >= 1.0 && r <= 8.0 && (e - r) < 1e-12 && (r - e) < 1e-12) ? (int)r : 0;
    }
};

// x^y in double as exp(y ln x) for y > 0, the powers of the gas constants
// the solver takes of positive ratios (a few ulp; x = 0 gives 0, x = inf
// gives inf, negative x or NaN give NaN):
//   ln x = e ln2 + 2 atanh(s), x = m 2^e, m in [1/sqrt2, sqrt2),
//   s = (m - 1)/(m + 1), |s| < 0.1716, atanh by its power series through
//   s^21 (the first omitted term is below 2^-55 of the sum);
//   exp t = 2^n exp(r), n = rint(t / ln2), r = t - n ln2 with ln2 split in a
//   33-bit head and a tail (Cody and Waite's reduction; n times the head is
//   exact for |n| < 2^20),
//   exp(r) by its Taylor series through r^13 (omitted part below 2^-56).
__device__ __forceinline__ double mm_pow(double x, double y) {
    constexpr double ln2_hi = 0x1.62e42fee00000p-1, ln2_lo = 0x1.a39ef35793c76p-33;
    int e;
    double m = frexp(x, &e);               // m in [1/2, 1)
    if (m < 0.70710678118654752440) { m *= 2.0; e -= 1; }
    const double sa = (m - 1.0) / (m + 1.0), z = sa * sa;
    double q = 1.0 / 21.0;
    q = fma(q, z, 1.0 / 19.0); q = fma(q, z, 1.0 / 17.0); q = fma(q, z, 1.0 / 15.0);
    q = fma(q, z, 1.0 / 13.0); q = fma(q, z, 1.0 / 11.0); q = fma(q, z, 1.0 / 9.0);
    q = fma(q, z, 1.0 / 7.0); q = fma(q, z, 1.0 / 5.0); q = fma(q, z, 1.0 / 3.0); q = fma(q, z, 1.0);
    const double de = (double)e;
    const double lnx = fma(de, ln2_hi, fma(de, ln2_lo, 2.0 * sa * q));
    const double t = y * lnx;
    const double n = rint(t * 1.44269504088896340736);
    const double r = fma(-n, ln2_lo, fma(-n, ln2_hi, t));
    double pe = 1.0 / 6227020800.0;         // 1/13!
    pe = fma(pe, r, 1.0 / 479001600.0); pe = fma(pe, r, 1.0 / 39916800.0); pe = fma(pe, r, 1.0 / 3628800.0);
    pe = fma(pe, r, 1.0 / 362880.0); pe = fma(pe, r, 1.0 / 40320.0); pe = fma(pe, r, 1.0 / 5040.0);
    pe = fma(pe, r, 1.0 / 720.0); pe = fma(pe, r, 1.0 / 120.0); pe = fma(pe, r, 1.0 / 24.0);
    pe = fma(pe, r, 1.0 / 6.0); pe = fma(pe, r, 0.5); pe = fma(pe, r, 1.0); pe = fma(pe, r, 1.0);
    const double res = ldexp(pe, (int)n);
    return x > 0.0 ? (x < (double)INFINITY ? res : x) : (x == 0.0 ? 0.0 : (double)NAN);
}
__device__ __forceinline__ float mm_pow(float x, float y) { return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x)); }
__device__ __forceinline__ double mm_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float mm_sqrt(float x) { return __builtin_sqrtf(x); }

// x^(2/(g-1)): multiplied out for integer exponents.
template <typename T> __device__ __forceinline__ T pow_rho(T x, const GasConst<T> &k) {
    if (k.iexp_rho > 0) {
        T r = x;
        for (int q = 1; q < k.iexp_rho; q++) r *= x;
        return r;
    }
    return mm_pow(x, k.exp_rho);
}

// One side of the Riemann problem with the constants of its pressure branch.
template <typename T> struct Side {
    T rho, u, P, c;
    T A, B;        // shock branch: A = 2/((g+1) rho), B = (g-1)/(g+1) P
    T fc;          // rarefaction branch prefactor 2c/(g-1)
    T inv_rc;      // 1/(rho c)
    T inv_P;
};

template <typename T>
__device__ __forceinline__ Side<T> make_side(T rho, T u, T P, const GasConst<T> &k) {
    Side<T> s;
    s.rho = rho; s.u = u; s.P = P;
    s.c = mm_sqrt(k.g * P / rho);
    s.A = k.two_over_gp1 / rho;
    s.B = k.gm_ratio * P;
    s.fc = k.two_over_gm1 * s.c;
    s.inv_rc = (T)1 / (rho * s.c);
    s.inv_P = (T)1 / P;
    return s;
}

// f_K(p) and f_K'(p); pw receives (p/p_K)^z on the isentropic branch.
template <typename T>
__device__ __forceinline__ void side_fn(T p, const Side<T> &s, const GasConst<T> &k, T &f, T &df, T &pw) {
    if (p > s.P) {
        T pb = p + s.B;
        T q = mm_sqrt(s.A / pb);
        f = (p - s.P) * q;
        df = q * ((T)1 - (T)0.5 * (p - s.P) / pb);
        pw = (T)-1;
    } else {
        T r = p * s.inv_P;
        pw = mm_pow(r, k.z);
        f = s.fc * (pw - (T)1);
        df = s.inv_rc * pw / r;
    }
}

// Adaptive non-iterative starting guess: the primitive-variable estimate
// when the pressure ratio is mild and it falls between the two pressures,
// else the two-rarefaction estimate (below) or the two-shock estimate (above).
// vac_num = c_L + c_R - (g-1)/2 (u_R - u_L): the vacuum test (vac_num <= 0)
// and the two-rarefaction estimate use this one value, so that a problem
// judged free of vacuum always has a positive two-rarefaction estimate.
template <typename T>
__device__ __forceinline__ T standard_guess(const Side<T> &L, const Side<T> &R, const GasConst<T> &k, T vac_num) {
    T du = R.u - L.u;
    T ppv = (T)0.5 * (L.P + R.P) - (T)0.125 * du * (L.rho + R.rho) * (L.c + R.c);
    ppv = ppv > (T)0 ? ppv : (T)0;
    T pmin = L.P < R.P ? L.P : R.P;
    T pmax = L.P < R.P ? R.P : L.P;
    if (pmax <= (T)2 * pmin && ppv >= pmin && ppv <= pmax) return ppv;
    if (ppv < pmin) {
        T den = L.c * mm_pow(L.inv_P, k.z) + R.c * mm_pow(R.inv_P, k.z);
        T ptr = mm_pow(vac_num / den, k.inv_z);
        return ptr > (T)0 ? ptr : (T)1e-30 * pmin;
    }
    T gL = mm_sqrt(L.A / (ppv + L.B));
    T gR = mm_sqrt(R.A / (ppv + R.B));
    T pts = (gL * L.P + gR * R.P - du) / (gL + gR);
    return pts > (T)0 ? pts : ppv;
}

// Result of the Newton iteration: the star state and the side powers
// (p*/p_K)^z of isentropic sides, for sampling.
template <typename T> struct Star {
    T ps, us, pwL, pwR;
    int iters;
    bool conv;
};

// Newton iteration on the pressure function, then u* = (u_L+u_R)/2 +
// (f_R(p*) - f_L(p*))/2. Converged when the relative step falls below tol or
// f(p) vanishes to within the rounding of its own terms (near vacuum the
// root can be ~1e-30 of the side pressures, where f' p is so small that
// rounding noise in f alone moves p by more than tol).
template <typename T>
__device__ __forceinline__ Star<T> newton_star(const Side<T> &L, const Side<T> &R, const GasConst<T> &k, T p,
                                               T tol, int maxit) {
    const T du = R.u - L.u;
    const T noise = (T)8 * (sizeof(T) == 8 ? (T)2.220446049250313e-16 : (T)1.1920929e-7);
    Star<T> st;
    st.iters = 0;
    st.conv = false;
    if (!(p > (T)0)) p = (T)0.5 * (L.P + R.P);
    T fl = 0, fr = 0, dfl = 1, dfr = 1, pwl = -1, pwr = -1, plast = p;
    while (st.iters < maxit) {
        side_fn(p, L, k, fl, dfl, pwl);
        side_fn(p, R, k, fr, dfr, pwr);
        const T fsum = fl + fr + du;
        T pn = p - fsum / (dfl + dfr);
        if (!(pn > (T)0)) pn = (T)0.1 * p;
        st.iters++;
        const bool done = fabs(pn - p) <= tol * (T)0.5 * (pn + p) ||
                          fabs(fsum) <= noise * (fabs(fl) + fabs(fr) + fabs(du));
        plast = p;
        p = pn;
        if (done) { st.conv = true; break; }
    }
    st.ps = p;
    const T dlt = p - plast;
    const bool small = fabs(dlt) <= (T)1e-6 * plast;
    if (small) {
        st.us = (T)0.5 * (L.u + R.u) + (T)0.5 * ((fr + dfr * dlt) - (fl + dfl * dlt));
    } else {
        T a, b, c2, d2, e1, e2;
        side_fn(p, L, k, a, b, e1);
        side_fn(p, R, k, c2, d2, e2);
        st.us = (T)0.5 * (L.u + R.u) + (T)0.5 * (c2 - a);
    }
    const T corr = (T)1 + k.z * dlt / plast;
    st.pwL = (p <= L.P) ? ((small && pwl > (T)0) ? pwl * corr : mm_pow(p * L.inv_P, k.z)) : (T)-1;
    st.pwR = (p <= R.P) ? ((small && pwr > (T)0) ? pwr * corr : mm_pow(p * R.inv_P, k.z)) : (T)-1;
    return st;
}

// Sampled face state; pstar is the star pressure and pstd the standard
// starting guess (both -1 where the problem has no star state, i.e.
// vacuum), filled by the caller of sample0.
template <typename T> struct FaceState { T rho, u, P; int side; T pstar, pstd; };

// Rarefaction fan of side K sampled at x/t = 0; `left` selects the
// characteristic family (u - c for the left state, u + c for the right).
// rho = rho_K (c/c_K)^(2/(g-1)), P = P_K (c/c_K)^(2g/(g-1)) = P_K (c/c_K)^(2/(g-1)) (c/c_K)^2.
template <typename T>
__device__ __forceinline__ FaceState<T> fan0(const Side<T> &K, bool left, const GasConst<T> &k) {
    FaceState<T> o;
    T c = left ? k.two_over_gp1 * (K.c + k.gm1_over_2 * K.u)
               : k.two_over_gp1 * (K.c - k.gm1_over_2 * K.u);
    T ratio = c / K.c;
    T pr = pow_rho(ratio, k);
    o.rho = K.rho * pr;
    o.u = left ? c : -c;
    o.P = K.P * pr * ratio * ratio;
    o.side = left ? 0 : 1;
    return o;
}

template <typename T>
__device__ __forceinline__ FaceState<T> undisturbed(const Side<T> &K, int side) {
    FaceState<T> o; o.rho = K.rho; o.u = K.u; o.P = K.P; o.side = side; return o;
}

template <typename T>
__device__ __forceinline__ FaceState<T> vac(int side) {
    FaceState<T> o; o.rho = (T)0; o.u = (T)0; o.P = (T)0; o.side = side; return o;
}

// Vacuum cases that need no star pressure. Returns true (and fills *o) if
// the problem is one of them; otherwise leaves vac_num for the guess.
template <typename T>
__device__ __forceinline__ bool vacuum_cases(const GasConst<T> &k, const Side<T> &L, const Side<T> &R, bool lvac,
                                             bool rvac, FaceState<T> &o, T &vac_num) {
    if (lvac && rvac) { o = vac<T>(0); return true; }
    if (lvac) {
        if ((T)0 >= R.u + R.c) o = undisturbed(R, 1);
        else if ((T)0 <= R.u - k.two_over_gm1 * R.c) o = vac<T>(1);
        else o = fan0(R, false, k);
        return true;
    }
    if (rvac) {
        if ((T)0 <= L.u - L.c) o = undisturbed(L, 0);
        else if ((T)0 >= L.u + k.two_over_gm1 * L.c) o = vac<T>(0);
        else o = fan0(L, true, k);
        return true;
    }
    vac_num = L.c + R.c - k.gm1_over_2 * (R.u - L.u);
    if (!(vac_num > (T)0)) {
        T frontL = L.u + k.two_over_gm1 * L.c;
        T frontR = R.u - k.two_over_gm1 * R.c;
        if ((T)0 <= frontL) o = ((T)0 <= L.u - L.c) ? undisturbed(L, 0) : fan0(L, true, k);
        else if ((T)0 >= frontR) o = ((T)0 >= R.u + R.c) ? undisturbed(R, 1) : fan0(R, false, k);
        else o = vac<T>(0);
        return true;
    }
    return false;
}

// Sample the solution with known star state at x/t = 0. s.pwK = (p*/p_K)^z
// on an isentropic side.
template <typename T>
__device__ __forceinline__ FaceState<T> sample0(const Side<T> &L, const Side<T> &R, const Star<T> &s,
                                                const GasConst<T> &k) {
    const T ps = s.ps, us = s.us;
    FaceState<T> o;
    o.u = us;
    o.P = ps;
    if ((T)0 <= us) {
        o.side = 0;
        if (ps > L.P) {
            T SL = L.u - L.c * mm_sqrt(k.zs1 * ps * L.inv_P + k.zs2);
            if ((T)0 <= SL) return undisturbed(L, 0);
            T r = ps * L.inv_P;
            o.rho = L.rho * (r + k.gm_ratio) / (k.gm_ratio * r + (T)1);
            return o;
        }
        if ((T)0 <= L.u - L.c) return undisturbed(L, 0);
        if ((T)0 >= us - L.c * s.pwL) {
            o.rho = L.rho * pow_rho(s.pwL, k);   // (p*/p_L)^(1/g) = ((p*/p_L)^z)^(2/(g-1))
            return o;
        }
        return fan0(L, true, k);
    }
    o.side = 1;
    if (ps > R.P) {
        T SR = R.u + R.c * mm_sqrt(k.zs1 * ps * R.inv_P + k.zs2);
        if ((T)0 >= SR) return undisturbed(R, 1);
        T r = ps * R.inv_P;
        o.rho = R.rho * (r + k.gm_ratio) / (k.gm_ratio * r + (T)1);
        return o;
    }
    if ((T)0 >= R.u + R.c) return undisturbed(R, 1);
    if ((T)0 <= us + R.c * s.pwR) {
        o.rho = R.rho * pow_rho(s.pwR, k);
        return o;
    }
    return fan0(R, false, k);
}

}  // namespace mm
