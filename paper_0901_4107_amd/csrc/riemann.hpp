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
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace mm {

enum RiemannCase : int { RC_NORMAL = 0, RC_LEFT_VACUUM = 1, RC_RIGHT_VACUUM = 2,
                         RC_VACUUM_GENERATED = 3, RC_BOTH_VACUUM = 4 };

template <typename T> struct GasConst {
    T g, gm1, gp1, z, inv_z, zs1, zs2, gm_ratio, inv_g, two_over_gm1, two_over_gp1,
      gm1_over_2, exp_rho, exp_P, g_over_gm1;
    __device__ __forceinline__ explicit GasConst(double gamma) {
        g = (T)gamma;
        gm1 = (T)(gamma - 1.0);
        gp1 = (T)(gamma + 1.0);
        z = (T)((gamma - 1.0) / (2.0 * gamma));
        inv_z = (T)(2.0 * gamma / (gamma - 1.0));
        zs1 = (T)((gamma + 1.0) / (2.0 * gamma));
        zs2 = (T)((gamma - 1.0) / (2.0 * gamma));
        gm_ratio = (T)((gamma - 1.0) / (gamma + 1.0));
        inv_g = (T)(1.0 / gamma);
        two_over_gm1 = (T)(2.0 / (gamma - 1.0));
        two_over_gp1 = (T)(2.0 / (gamma + 1.0));
        gm1_over_2 = (T)(0.5 * (gamma - 1.0));
        exp_rho = (T)(2.0 / (gamma - 1.0));
        exp_P = (T)(2.0 * gamma / (gamma - 1.0));
        g_over_gm1 = (T)(gamma / (gamma - 1.0));
    }
};

__device__ __forceinline__ double mm_pow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float mm_pow(float x, float y) { return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x)); }
__device__ __forceinline__ double mm_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float mm_sqrt(float x) { return __builtin_sqrtf(x); }

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

template <typename T>
__device__ __forceinline__ void side_fn(T p, const Side<T> &s, const GasConst<T> &k, T &f, T &df) {
    if (p > s.P) {
        T pb = p + s.B;
        T q = mm_sqrt(s.A / pb);
        f = (p - s.P) * q;
        df = q * ((T)1 - (T)0.5 * (p - s.P) / pb);
    } else {
        T r = p * s.inv_P;
        T pw = mm_pow(r, k.z);
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

// Newton iteration on the pressure function. Returns the iteration count;
// *conv tells whether it converged: the relative step fell below tol, or
// f(p) vanished to within the rounding of its own terms (near vacuum the
// root can be ~1e-30 of the side pressures, where f' p is so small that
// rounding noise in f alone moves p by more than tol).
template <typename T>
__device__ __forceinline__ int newton_star(const Side<T> &L, const Side<T> &R, const GasConst<T> &k,
                                           T p, T tol, int maxit, T &pstar, bool &conv) {
    T du = R.u - L.u;
    int it = 0;
    conv = false;
    if (!(p > (T)0)) p = (T)0.5 * (L.P + R.P);
    const T noise = (T)8 * (sizeof(T) == 8 ? (T)2.220446049250313e-16 : (T)1.1920929e-7);
    while (it < maxit) {
        T fl, dfl, fr, dfr;
        side_fn(p, L, k, fl, dfl);
        side_fn(p, R, k, fr, dfr);
        const T fsum = fl + fr + du;
        T pn = p - fsum / (dfl + dfr);
        if (!(pn > (T)0)) pn = (T)0.1 * p;
        it++;
        bool done = fabs(pn - p) <= tol * (T)0.5 * (pn + p) ||
                    fabs(fsum) <= noise * (fabs(fl) + fabs(fr) + fabs(du));
        p = pn;
        if (done) { conv = true; break; }
    }
    pstar = p;
    return it;
}

template <typename T> struct FaceState { T rho, u, P; int side; };

// Rarefaction fan of side K sampled at x/t = 0; `left` selects the
// characteristic family (u - c for the left state, u + c for the right).
template <typename T>
__device__ __forceinline__ FaceState<T> fan0(const Side<T> &K, bool left, const GasConst<T> &k) {
    FaceState<T> o;
    T c = left ? k.two_over_gp1 * (K.c + k.gm1_over_2 * K.u)
               : k.two_over_gp1 * (K.c - k.gm1_over_2 * K.u);
    T ratio = c / K.c;
    o.rho = K.rho * mm_pow(ratio, k.exp_rho);
    o.u = left ? c : -c;
    o.P = K.P * mm_pow(ratio, k.exp_P);
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
// the problem is one of them.
template <typename T>
__device__ __forceinline__ bool vacuum_cases(T rhoL, T uL, T PL, T rhoR, T uR, T PR, const GasConst<T> &k,
                                             const Side<T> &L, const Side<T> &R, bool lvac, bool rvac,
                                             FaceState<T> &o, int &kase, T &vac_num) {
    if (lvac && rvac) { o = vac<T>(0); kase = RC_BOTH_VACUUM; return true; }
    if (lvac) {
        kase = RC_LEFT_VACUUM;
        if ((T)0 >= R.u + R.c) o = undisturbed(R, 1);
        else if ((T)0 <= R.u - k.two_over_gm1 * R.c) o = vac<T>(1);
        else o = fan0(R, false, k);
        return true;
    }
    if (rvac) {
        kase = RC_RIGHT_VACUUM;
        if ((T)0 <= L.u - L.c) o = undisturbed(L, 0);
        else if ((T)0 >= L.u + k.two_over_gm1 * L.c) o = vac<T>(0);
        else o = fan0(L, true, k);
        return true;
    }
    vac_num = L.c + R.c - k.gm1_over_2 * (R.u - L.u);
    if (!(vac_num > (T)0)) {
        kase = RC_VACUUM_GENERATED;
        T frontL = L.u + k.two_over_gm1 * L.c;
        T frontR = R.u - k.two_over_gm1 * R.c;
        if ((T)0 <= frontL) o = ((T)0 <= L.u - L.c) ? undisturbed(L, 0) : fan0(L, true, k);
        else if ((T)0 >= frontR) o = ((T)0 >= R.u + R.c) ? undisturbed(R, 1) : fan0(R, false, k);
        else o = vac<T>(0);
        return true;
    }
    return false;
}

// Sample the solution with known star state at x/t = 0.
template <typename T>
__device__ __forceinline__ FaceState<T> sample0(const Side<T> &L, const Side<T> &R, T ps, T us,
                                                const GasConst<T> &k) {
    if ((T)0 <= us) {
        if (ps > L.P) {
            T SL = L.u - L.c * mm_sqrt(k.zs1 * ps * L.inv_P + k.zs2);
            if ((T)0 <= SL) return undisturbed(L, 0);
            T r = ps * L.inv_P;
            FaceState<T> o; o.rho = L.rho * (r + k.gm_ratio) / (k.gm_ratio * r + (T)1); o.u = us; o.P = ps; o.side = 0;
            return o;
        }
        if ((T)0 <= L.u - L.c) return undisturbed(L, 0);
        T r = ps * L.inv_P;
        T cs = L.c * mm_pow(r, k.z);
        if ((T)0 >= us - cs) {
            FaceState<T> o; o.rho = L.rho * mm_pow(r, k.inv_g); o.u = us; o.P = ps; o.side = 0;
            return o;
        }
        return fan0(L, true, k);
    }
    if (ps > R.P) {
        T SR = R.u + R.c * mm_sqrt(k.zs1 * ps * R.inv_P + k.zs2);
        if ((T)0 >= SR) return undisturbed(R, 1);
        T r = ps * R.inv_P;
        FaceState<T> o; o.rho = R.rho * (r + k.gm_ratio) / (k.gm_ratio * r + (T)1); o.u = us; o.P = ps; o.side = 1;
        return o;
    }
    if ((T)0 >= R.u + R.c) return undisturbed(R, 1);
    T r = ps * R.inv_P;
    T cs = R.c * mm_pow(r, k.z);
    if ((T)0 <= us + cs) {
        FaceState<T> o; o.rho = R.rho * mm_pow(r, k.inv_g); o.u = us; o.P = ps; o.side = 1;
        return o;
    }
    return fan0(R, false, k);
}

// u* from the converged star pressure.
template <typename T>
__device__ __forceinline__ T star_velocity(const Side<T> &L, const Side<T> &R, T ps, const GasConst<T> &k) {
    T fl, dfl, fr, dfr;
    side_fn(ps, L, k, fl, dfl);
    side_fn(ps, R, k, fr, dfr);
    return (T)0.5 * (L.u + R.u) + (T)0.5 * (fr - fl);
}

}  // namespace mm
