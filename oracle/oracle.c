/*
 * oracle.c -- plain, slow, double-precision CPU reference for one
 * finite-volume hydro step of the moving Voronoi-mesh Godunov scheme
 * (Springel, "E pur si muove", arXiv:0901.4107, Section 3).
 *
 * TEST INFRASTRUCTURE. This file is the checker, not the product: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it. It shares no source with the GPU library and includes none of its
 * headers. Every function names the passage of the paper it follows; where
 * the paper is silent the reading taken is stated in the comment.
 *
 * Layouts (identical to the public ABI so that tests can pass the same
 * arrays to both sides, but re-declared here on purpose):
 *   conserved  Q [D+2][N]  rows m, p_x, p_y(, p_z), E      (cell totals);
 *              [D+3][N] with the total entropy S as last row (Section 3.5)
 *   primitive  W [D+2][N]  rows rho, v_x, v_y(, v_z), P
 *   gradient   G [D+2][D][N]  G[(c*D + k)*N + i] = d W_c / d x_k in cell i
 *   per-face vectors [D][F]; per-cell vectors [D][N]
 *   face_ctr   g = f - r_L  (face centroid relative to the left generator)
 *   face_sep   d = r_R - r_L (periodic image of R as seen from L)
 *   centroid_off  delta_i = s_i - r_i
 * The face normal points from L to R.
 *
 * Threads: the loops of the step run on the host's cores (OpenMP). Each
 * parallel loop treats independent faces or cells; where the plain method
 * scatters face terms into cells (gradients, the update), each cell instead
 * gathers its faces' terms in ascending face order, which is the order in
 * which a single loop over the faces adds them, so the results are the same
 * bit for bit for any number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI_D 3.14159265358979323846

typedef struct {
    int32_t dim;
    int64_t n_cells, n_faces;
    const double *volume;       /* [N] */
    const double *centroid_off; /* [D][N] s_i - r_i */
    const double *mesh_vel;     /* [D][N] w_i */
    const int32_t *face_L, *face_R; /* [F] */
    const double *face_area;    /* [F] */
    const double *face_ctr;     /* [D][F] f - r_L */
    const double *face_sep;     /* [D][F] r_R - r_L */
} om_mesh;

typedef struct {
    double gamma;
    double cfl;
} om_params;

/* Number of host threads for the loops below (1 without OpenMP). */
void oracle_set_threads(int32_t n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int32_t oracle_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* The faces of every cell in ascending face order: cell i has the faces
 * face[off[i] .. off[i+1]-1], right[q] = 1 where i is the face's right cell.
 * A counting sort over the face list, in one plain loop. */
typedef struct {
    int64_t *off;
    int32_t *face;
    int8_t *right;
} om_sides;

static void sides_build(const om_mesh *M, om_sides *S)
{
    const int64_t n = M->n_cells, nf = M->n_faces;
    S->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    S->face = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)nf);
    S->right = (int8_t *)malloc(2 * (size_t)nf);
    for (int64_t f = 0; f < nf; f++) {
        S->off[M->face_L[f] + 1]++;
        S->off[M->face_R[f] + 1]++;
    }
    for (int64_t i = 0; i < n; i++) S->off[i + 1] += S->off[i];
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    memcpy(next, S->off, sizeof(int64_t) * (size_t)n);
    for (int64_t f = 0; f < nf; f++) {
        int64_t q = next[M->face_L[f]]++;
        S->face[q] = (int32_t)f;
        S->right[q] = 0;
        q = next[M->face_R[f]]++;
        S->face[q] = (int32_t)f;
        S->right[q] = 1;
    }
    free(next);
}

static void sides_free(om_sides *S)
{
    free(S->off); free(S->face); free(S->right);
}

/* ------------------------------------------------------------------ */
/* Exact Riemann solver for the 1D Euler equations of an ideal gas.      */
/* Section 3.3 (flux computation) names an exact solver with a vacuum    */
/* extension; the wave structure below is the textbook exact solution:   */
/* two nonlinear waves (shock or rarefaction) around a contact, the star */
/* pressure being the root of the pressure function                      */
/*   f(p) = f_L(p) + f_R(p) + (u_R - u_L).                               */
/* ------------------------------------------------------------------ */

enum { OR_NORMAL = 0, OR_LEFT_VACUUM = 1, OR_RIGHT_VACUUM = 2,
       OR_VACUUM_GENERATED = 3, OR_BOTH_VACUUM = 4 };

/* One side's contribution f_K(p) to the pressure function and its
 * derivative. Shock branch (p > p_K): Rankine-Hugoniot relation; rarefaction
 * branch (p <= p_K): isentropic relation with the generalised Riemann
 * invariant. */
static void pressure_side(double p, double rho, double P, double c, double g,
                          double *f, double *df)
{
    if (p > P) {
        double Ak = 2.0 / ((g + 1.0) * rho);
        double Bk = (g - 1.0) / (g + 1.0) * P;
        double q = sqrt(Ak / (p + Bk));
        *f = (p - P) * q;
        *df = q * (1.0 - 0.5 * (p - P) / (p + Bk));
    } else {
        double z = (g - 1.0) / (2.0 * g);
        double ratio = p / P;
        *f = 2.0 * c / (g - 1.0) * (pow(ratio, z) - 1.0);
        /* d/dp of the above = (1/(rho c)) (p/P)^(-(g+1)/(2g)) */
        *df = (p > 0.0) ? pow(ratio, -(g + 1.0) / (2.0 * g)) / (rho * c) : INFINITY;
    }
}

static double pressure_function(double p, const double *L, const double *R,
                                double cL, double cR, double g, double *dfdp)
{
    double fl, dfl, fr, dfr;
    pressure_side(p, L[0], L[2], cL, g, &fl, &dfl);
    pressure_side(p, R[0], R[2], cR, g, &fr, &dfr);
    if (dfdp) *dfdp = dfl + dfr;
    return fl + fr + (R[1] - L[1]);
}

/* Root of the (monotone increasing, concave) pressure function, found by
 * Newton's method kept inside a bisection bracket [lo, hi] with
 * f(lo) < 0 < f(hi). Runs until the step is within 4 ulp of p. Returns the
 * number of iterations. */
static int star_pressure(const double *L, const double *R, double cL, double cR,
                         double g, double *pstar)
{
    double lo = 0.0;
    double hi = fmax(L[2], R[2]);
    int guard = 0;
    while (pressure_function(hi, L, R, cL, cR, g, NULL) <= 0.0 && guard < 2000) {
        hi *= 2.0;
        guard++;
    }
    double p = 0.5 * (L[2] + R[2]);
    if (!(p > lo && p < hi)) p = 0.5 * (lo + hi);
    int it;
    for (it = 1; it <= 400; it++) {
        double df;
        double f = pressure_function(p, L, R, cL, cR, g, &df);
        if (f == 0.0) break;
        if (f < 0.0) lo = p; else hi = p;
        double pn = p - f / df;
        /* a Newton step below 4 ulp that stays in the closed bracket ends
         * the search (the step may round to p itself) */
        if (fabs(pn - p) <= 4.0 * DBL_EPSILON * p && pn >= lo && pn <= hi) { p = pn; break; }
        if (!(pn > lo && pn < hi)) pn = 0.5 * (lo + hi);
        p = pn;
        if (hi - lo <= 4.0 * DBL_EPSILON * hi) break;
    }
    *pstar = p;
    return it;
}

/* Sample the rarefaction fan of the left (sign=+1) or right (sign=-1)
 * state at x/t = S: the characteristic u -/+ c = S meets the Riemann
 * invariant u +/- 2c/(g-1) carried from the undisturbed side. */
static void sample_fan(const double *K, double cK, double g, double S, int left,
                       double *out)
{
    double c;
    if (left)
        c = 2.0 / (g + 1.0) * (cK + 0.5 * (g - 1.0) * (K[1] - S));
    else
        c = 2.0 / (g + 1.0) * (cK - 0.5 * (g - 1.0) * (K[1] - S));
    double ratio = c / cK;
    out[0] = K[0] * pow(ratio, 2.0 / (g - 1.0));
    out[1] = left ? S + c : S - c;
    out[2] = K[2] * pow(ratio, 2.0 * g / (g - 1.0));
}

/*
 * Solve the Riemann problem with left state L=(rho,u,P), right state R and
 * sample it at x/t = 0 (Section 3.3). out[0..2] = (rho_F, u_F, P_F) and
 * out[3] = 0 if the sample lies on the left-state side of the contact
 * (whose transverse velocity is then upwind), 1 if on the right side.
 * star[0..1] = (p*, u*) where defined (NaN otherwise); *iters = iterations of
 * the root finder (0 if not run). A side with rho <= 0 or P <= 0 is taken as
 * vacuum. Returns the case code.
 */
int oracle_riemann(double g, const double *Lin, const double *Rin,
                   double *out, double *star, int *iters)
{
    double L[3] = {Lin[0], Lin[1], Lin[2]};
    double R[3] = {Rin[0], Rin[1], Rin[2]};
    const double S = 0.0;
    int lvac = !(L[0] > 0.0 && L[2] > 0.0);
    int rvac = !(R[0] > 0.0 && R[2] > 0.0);
    star[0] = NAN; star[1] = NAN;
    if (iters) *iters = 0;

    if (lvac && rvac) {
        out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; out[3] = 0.0;
        return OR_BOTH_VACUUM;
    }
    if (lvac) {
        /* right state next to vacuum: a left-facing fan ending at the
         * vacuum front u_R - 2 c_R/(g-1) */
        double cR = sqrt(g * R[2] / R[0]);
        double head = R[1] + cR;
        double front = R[1] - 2.0 * cR / (g - 1.0);
        out[3] = 1.0;
        if (S >= head) { out[0] = R[0]; out[1] = R[1]; out[2] = R[2]; }
        else if (S <= front) { out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; }
        else sample_fan(R, cR, g, S, 0, out);
        return OR_LEFT_VACUUM;
    }
    if (rvac) {
        double cL = sqrt(g * L[2] / L[0]);
        double head = L[1] - cL;
        double front = L[1] + 2.0 * cL / (g - 1.0);
        out[3] = 0.0;
        if (S <= head) { out[0] = L[0]; out[1] = L[1]; out[2] = L[2]; }
        else if (S >= front) { out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; }
        else sample_fan(L, cL, g, S, 1, out);
        return OR_RIGHT_VACUUM;
    }

    double cL = sqrt(g * L[2] / L[0]);
    double cR = sqrt(g * R[2] / R[0]);
    if (R[1] - L[1] >= 2.0 * (cL + cR) / (g - 1.0)) {
        /* the two rarefactions do not meet: vacuum opens between them */
        double frontL = L[1] + 2.0 * cL / (g - 1.0);
        double frontR = R[1] - 2.0 * cR / (g - 1.0);
        if (S <= frontL) {
            out[3] = 0.0;
            if (S <= L[1] - cL) { out[0] = L[0]; out[1] = L[1]; out[2] = L[2]; }
            else sample_fan(L, cL, g, S, 1, out);
        } else if (S >= frontR) {
            out[3] = 1.0;
            if (S >= R[1] + cR) { out[0] = R[0]; out[1] = R[1]; out[2] = R[2]; }
            else sample_fan(R, cR, g, S, 0, out);
        } else {
            out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; out[3] = 0.0;
        }
        return OR_VACUUM_GENERATED;
    }

    double ps;
    int it = star_pressure(L, R, cL, cR, g, &ps);
    if (iters) *iters = it;
    double fl, dfl, fr, dfr;
    pressure_side(ps, L[0], L[2], cL, g, &fl, &dfl);
    pressure_side(ps, R[0], R[2], cR, g, &fr, &dfr);
    double us = 0.5 * (L[1] + R[1]) + 0.5 * (fr - fl);
    star[0] = ps; star[1] = us;

    double gm = (g - 1.0) / (g + 1.0);
    if (S <= us) {
        out[3] = 0.0;
        if (ps > L[2]) {
            double SL = L[1] - cL * sqrt((g + 1.0) / (2.0 * g) * ps / L[2] + (g - 1.0) / (2.0 * g));
            if (S <= SL) { out[0] = L[0]; out[1] = L[1]; out[2] = L[2]; }
            else {
                double r = ps / L[2];
                out[0] = L[0] * (r + gm) / (gm * r + 1.0);
                out[1] = us; out[2] = ps;
            }
        } else {
            double head = L[1] - cL;
            double cs = cL * pow(ps / L[2], (g - 1.0) / (2.0 * g));
            double tail = us - cs;
            if (S <= head) { out[0] = L[0]; out[1] = L[1]; out[2] = L[2]; }
            else if (S >= tail) {
                out[0] = L[0] * pow(ps / L[2], 1.0 / g);
                out[1] = us; out[2] = ps;
            } else sample_fan(L, cL, g, S, 1, out);
        }
    } else {
        out[3] = 1.0;
        if (ps > R[2]) {
            double SR = R[1] + cR * sqrt((g + 1.0) / (2.0 * g) * ps / R[2] + (g - 1.0) / (2.0 * g));
            if (S >= SR) { out[0] = R[0]; out[1] = R[1]; out[2] = R[2]; }
            else {
                double r = ps / R[2];
                out[0] = R[0] * (r + gm) / (gm * r + 1.0);
                out[1] = us; out[2] = ps;
            }
        } else {
            double head = R[1] + cR;
            double cs = cR * pow(ps / R[2], (g - 1.0) / (2.0 * g));
            double tail = us + cs;
            if (S >= head) { out[0] = R[0]; out[1] = R[1]; out[2] = R[2]; }
            else if (S <= tail) {
                out[0] = R[0] * pow(ps / R[2], 1.0 / g);
                out[1] = us; out[2] = ps;
            } else sample_fan(R, cR, g, S, 0, out);
        }
    }
    return OR_NORMAL;
}

/* Batched form for the tests: arrays of n problems. */
void oracle_riemann_batch(int64_t n, double g,
                          const double *rhoL, const double *uL, const double *PL,
                          const double *rhoR, const double *uR, const double *PR,
                          double *rhoF, double *uF, double *PF, double *side,
                          double *pstar, double *ustar, int32_t *kase, int32_t *iters)
{
    for (int64_t i = 0; i < n; i++) {
        double L[3] = {rhoL[i], uL[i], PL[i]};
        double R[3] = {rhoR[i], uR[i], PR[i]};
        double out[4], st[2];
        int it;
        int k = oracle_riemann(g, L, R, out, st, &it);
        rhoF[i] = out[0]; uF[i] = out[1]; PF[i] = out[2]; side[i] = out[3];
        pstar[i] = st[0]; ustar[i] = st[1];
        if (kase) kase[i] = k;
        if (iters) iters[i] = it;
    }
}

/* The pressure function itself, exposed so that tests can check that a
 * returned p* is a root (f(p*) = 0) independently of the solver loop. */
double oracle_pressure_function(double g, const double *L, const double *R, double p)
{
    double cL = sqrt(g * L[2] / L[0]);
    double cR = sqrt(g * R[2] / R[0]);
    return pressure_function(p, L, R, cL, cR, g, NULL);
}

/* ------------------------------------------------------------------ */
/* Step (ii): conserved -> primitive (Section 3, state vector and EOS).  */
/* rho = m/V, v = p/m, P = (g-1)(E - m v^2/2)/V. A cell with m <= 0 is   */
/* vacuum: all primitives zero.                                          */
/* ------------------------------------------------------------------ */
void oracle_prim(int32_t dim, int64_t n, double g, const double *V,
                 const double *Q, double *W)
{
    const int nv = dim + 2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double m = Q[0 * n + i];
        double E = Q[(nv - 1) * n + i];
        if (!(m > 0.0)) {
            for (int c = 0; c < nv; c++) W[c * n + i] = 0.0;
            continue;
        }
        double ke = 0.0;
        W[0 * n + i] = m / V[i];
        for (int k = 0; k < dim; k++) {
            double v = Q[(1 + k) * n + i] / m;
            W[(1 + k) * n + i] = v;
            ke += v * v;
        }
        W[(nv - 1) * n + i] = (g - 1.0) * (E - 0.5 * m * ke) / V[i];
    }
}

/* ------------------------------------------------------------------ */
/* Step (iii): gradients and slope limiting (Section 3.1).               */
/* Gradient: the Voronoi estimate exact to linear order,                 */
/*   V_i grad phi_i = sum_j A_ij ( [phi_j - phi_i] c_ij / r_ij           */
/*                                 - (phi_i + phi_j)/2 * r_ij / r_ij ),  */
/* with r_ij = r_i - r_j and c_ij = f_ij - (r_i + r_j)/2. Written per     */
/* face from the left cell's view (r_LR = -d, c = g - d/2); the right     */
/* cell's term is the negative because A, c and |r| are symmetric while   */
/* r_ij flips sign. Accumulated per cell in face-list order.             */
/* Limiter: alpha_i = min(1, min_j psi_ij) per primitive, with the        */
/* neighbour extrema taken over the face neighbours and i itself, and    */
/* Delta phi_ij = grad phi_i . (f_ij - s_i). A |Delta phi| at round-off   */
/* level (<= 1e-13 max(|phi_i|, phi_max - phi_min)) is read as zero.      */
/* ------------------------------------------------------------------ */
static void gradients_with(const om_mesh *M, const om_sides *S, const double *W, double *grad_raw,
                           double *grad_lim, double *alpha)
{
    const int D = M->dim, nv = D + 2;
    const int64_t n = M->n_cells, nf = M->n_faces;
    const double *A = M->face_area, *gc = M->face_ctr, *ds = M->face_sep;

#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double acc[5][3] = {{0}}, phimin[5], phimax[5];
        for (int c = 0; c < nv; c++) { phimin[c] = W[c * n + i]; phimax[c] = W[c * n + i]; }
        /* the face terms of cell i, from the left cell's view: + on the
           left cell, - on the right one */
        for (int64_t q = S->off[i]; q < S->off[i + 1]; q++) {
            const int64_t f = S->face[q];
            const int right = S->right[q];
            const int64_t l = M->face_L[f], r = M->face_R[f];
            double d[3] = {0, 0, 0}, cc[3] = {0, 0, 0}, ell = 0.0;
            for (int k = 0; k < D; k++) { d[k] = ds[k * nf + f]; ell += d[k] * d[k]; }
            ell = sqrt(ell);
            for (int k = 0; k < D; k++) cc[k] = gc[k * nf + f] - 0.5 * d[k];
            for (int c = 0; c < nv; c++) {
                double pl = W[c * n + l], pr = W[c * n + r];
                for (int k = 0; k < D; k++) {
                    double G = A[f] / ell * ((pr - pl) * cc[k] + 0.5 * (pl + pr) * d[k]);
                    if (right) acc[c][k] -= G;
                    else acc[c][k] += G;
                }
                double other = right ? pl : pr;
                if (other < phimin[c]) phimin[c] = other;
                if (other > phimax[c]) phimax[c] = other;
            }
        }
        for (int c = 0; c < nv; c++)
            for (int k = 0; k < D; k++)
                grad_raw[(c * D + k) * n + i] = acc[c][k] / M->volume[i];

        /* limiter: every face of cell i */
        double al[5] = {1.0, 1.0, 1.0, 1.0, 1.0};
        for (int64_t q = S->off[i]; q < S->off[i + 1]; q++) {
            const int64_t f = S->face[q];
            const int s = S->right[q];
            double dx[3] = {0, 0, 0};
            for (int k = 0; k < D; k++) {
                /* f - s_i: for L, g - delta_L; for R, g - d - delta_R */
                double fr = gc[k * nf + f] - (s ? ds[k * nf + f] : 0.0);
                dx[k] = fr - M->centroid_off[k * n + i];
            }
            for (int c = 0; c < nv; c++) {
                double phi = W[c * n + i];
                double dphi = 0.0;
                for (int k = 0; k < D; k++) dphi += grad_raw[(c * D + k) * n + i] * dx[k];
                double range = phimax[c] - phimin[c];
                double tol = 1e-13 * fmax(fabs(phi), range);
                double psi;
                if (dphi > tol) psi = (phimax[c] - phi) / dphi;
                else if (dphi < -tol) psi = (phimin[c] - phi) / dphi;
                else psi = 1.0;
                if (psi < al[c]) al[c] = psi;
            }
        }
        for (int c = 0; c < nv; c++) {
            for (int k = 0; k < D; k++)
                grad_lim[(c * D + k) * n + i] = al[c] * grad_raw[(c * D + k) * n + i];
            if (alpha) alpha[c * n + i] = al[c];
        }
    }
}

void oracle_gradients(const om_mesh *M, const double *W, double *grad_raw,
                      double *grad_lim, double *alpha)
{
    om_sides S;
    sides_build(M, &S);
    gradients_with(M, &S, W, grad_raw, grad_lim, alpha);
    sides_free(&S);
}

/* ------------------------------------------------------------------ */
/* Face velocity (Section 3.3, motion of the face centroid): the mean of */
/* the two generator velocities plus the normal motion of the centroid   */
/* induced by their residual motion,                                     */
/*   w = (w_L + w_R)/2 + [(w_L - w_R) . (f - (r_L+r_R)/2) / |d|] d/|d|.  */
/* ------------------------------------------------------------------ */
void oracle_face_velocity(const om_mesh *M, double *wf)
{
    const int D = M->dim;
    const int64_t n = M->n_cells, nf = M->n_faces;
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < nf; f++) {
        int64_t l = M->face_L[f], r = M->face_R[f];
        double d[3] = {0, 0, 0}, cc[3] = {0, 0, 0}, ell2 = 0.0, proj = 0.0;
        for (int k = 0; k < D; k++) {
            d[k] = M->face_sep[k * nf + f];
            cc[k] = M->face_ctr[k * nf + f] - 0.5 * d[k];
            ell2 += d[k] * d[k];
        }
        for (int k = 0; k < D; k++)
            proj += (M->mesh_vel[k * n + l] - M->mesh_vel[k * n + r]) * cc[k];
        for (int k = 0; k < D; k++)
            wf[k * nf + f] = 0.5 * (M->mesh_vel[k * n + l] + M->mesh_vel[k * n + r])
                             + proj * d[k] / ell2;
    }
}

/* ------------------------------------------------------------------ */
/* Step (vi): the flux across every face (Section 3.3).                  */
/* For each side K: go to the face rest frame (v' = v - w), extrapolate  */
/* to the face centroid with the limited gradient about the cell's       */
/* centre of mass and half a step forward in time with the primitive     */
/* Euler equations dW/dt = -A(W) grad W (evaluated at the cell's face-   */
/* frame state); split the velocity into the component along the unit   */
/* normal n = d/|d| and the transverse rest (the rotation Lambda only    */
/* needs that split); solve the Riemann problem and sample x/t = 0; use   */
/* the transverse velocity of the side the sample came from; form the    */
/* moving-face flux and return to the lab frame:                         */
/*   m_f = rho_F u_F,  Pi = m_f v_F + P_F n,                             */
/*   eps = m_f |v_F|^2/2 + u_F P_F g/(g-1),                              */
/*   lab flux = (m_f, Pi + m_f w, eps + Pi.w + m_f |w|^2/2).             */
/* If an extrapolated density or pressure is not positive on either     */
/* side, both sides use their unextrapolated face-frame cell states      */
/* (a reading: the paper does not treat this case).                      */
/* face_flux[c][f] = dt * A_f * Fhat_c. fallback[f] = 1 if that happened. */
/* ------------------------------------------------------------------ */
static void half_step(int D, double g, double dt, const double *Wc, const double grad[5][3],
                      const double *dx, double *out)
{
    /* Wc: rho, v'[D], P in the face frame; grad[c][k] = d W_c/d x_k */
    const int nv = D + 2;
    double rho = Wc[0], P = Wc[nv - 1];
    double div = 0.0;
    for (int k = 0; k < D; k++) div += grad[1 + k][k];
    double s, t;
    /* density */
    s = 0.0; t = 0.0;
    for (int k = 0; k < D; k++) { s += grad[0][k] * dx[k]; t += Wc[1 + k] * grad[0][k]; }
    out[0] = rho + s - 0.5 * dt * (t + rho * div);
    /* velocity */
    for (int i = 0; i < D; i++) {
        s = 0.0; t = 0.0;
        for (int k = 0; k < D; k++) { s += grad[1 + i][k] * dx[k]; t += Wc[1 + k] * grad[1 + i][k]; }
        out[1 + i] = Wc[1 + i] + s - 0.5 * dt * (t + grad[nv - 1][i] / rho);
    }
    /* pressure */
    s = 0.0; t = 0.0;
    for (int k = 0; k < D; k++) { s += grad[nv - 1][k] * dx[k]; t += Wc[1 + k] * grad[nv - 1][k]; }
    out[nv - 1] = P + s - 0.5 * dt * (t + g * P * div);
}

/* The face-frame Riemann inputs of every face (after extrapolation and the
 * positivity fallback): states[0..5][f] = rho_L, u_L, P_L, rho_R, u_R, P_R
 * with u the velocity component along the L->R normal. For tests. */
void oracle_face_states(const om_mesh *M, const om_params *prm, double dt,
                        const double *W, const double *grad, double *states)
{
    const int D = M->dim, nv = D + 2;
    const int64_t n = M->n_cells, nf = M->n_faces;
    double *wf = (double *)malloc(sizeof(double) * D * nf);
    oracle_face_velocity(M, wf);
    for (int64_t f = 0; f < nf; f++) {
        int64_t cell[2] = {M->face_L[f], M->face_R[f]};
        double d[3] = {0, 0, 0}, w[3] = {0, 0, 0}, ell = 0.0;
        for (int k = 0; k < D; k++) { d[k] = M->face_sep[k * nf + f]; ell += d[k] * d[k]; w[k] = wf[k * nf + f]; }
        ell = sqrt(ell);
        double Wp[2][5], Wpp[2][5];
        for (int s = 0; s < 2; s++) {
            int64_t i = cell[s];
            double dx[3] = {0, 0, 0}, gr[5][3];
            for (int k = 0; k < D; k++)
                dx[k] = M->face_ctr[k * nf + f] - (s ? d[k] : 0.0) - M->centroid_off[k * n + i];
            Wp[s][0] = W[0 * n + i];
            for (int k = 0; k < D; k++) Wp[s][1 + k] = W[(1 + k) * n + i] - w[k];
            Wp[s][nv - 1] = W[(nv - 1) * n + i];
            for (int c = 0; c < nv; c++)
                for (int k = 0; k < D; k++) gr[c][k] = grad[(c * D + k) * n + i];
            half_step(D, prm->gamma, dt, Wp[s], gr, dx, Wpp[s]);
        }
        int fb = !(Wpp[0][0] > 0.0 && Wpp[0][nv - 1] > 0.0 && Wpp[1][0] > 0.0 && Wpp[1][nv - 1] > 0.0);
        if (fb) memcpy(Wpp, Wp, sizeof(Wp));
        for (int s = 0; s < 2; s++) {
            double u = 0.0;
            for (int k = 0; k < D; k++) u += Wpp[s][1 + k] * d[k] / ell;
            states[(3 * s + 0) * nf + f] = Wpp[s][0];
            states[(3 * s + 1) * nf + f] = u;
            states[(3 * s + 2) * nf + f] = Wpp[s][nv - 1];
        }
    }
    free(wf);
}

/* Section 3.5 (poorly resolved cold flows), per face:
 *   entropy flux  m_F A_U with A_U = P_U / rho_U^g the entropic function of
 *                 the upwind side of the Riemann problem, the side the
 *                 solution at the face is sampled from (the sign of the
 *                 normal face velocity selects it); zero mass flux gives zero;
 *   shock Mach    for a side K whose pressure the star pressure exceeds (a
 *                 shock moves into K), the shock speed relative to the
 *                 unshocked gas over c_K, sqrt((g+1)/(2g) p* / p_K + (g-1)/(2g)).
 *                 Reading: the same expression is taken on both sides (on a
 *                 rarefied side it is below 1), so that the face value, the
 *                 larger of the two, is continuous where p* crosses p_K and
 *                 round-off there cannot switch it between 0 and 1; it is the
 *                 strongest shock's Mach number whenever that exceeds 1, and
 *                 0 for the vacuum cases (no star state).
 * s_flux [F] receives dt A m_F A_U, mach [F] the Mach number (both may be
 * NULL). */
void oracle_face_fluxes_ex(const om_mesh *M, const om_params *prm, double dt,
                           const double *W, const double *grad, double *face_flux,
                           int32_t *fallback, int32_t *kase, double *s_flux, double *mach);
void oracle_face_fluxes_full(const om_mesh *M, const om_params *prm, double dt, const double *accel,
                             const double *W, const double *grad, double *face_flux,
                             int32_t *fallback, int32_t *kase, double *s_flux, double *mach);

/* The face rule for the Mach number, given the Riemann case and p*. */
static double riemann_shock_mach(double g, const double *L, const double *R, int kase, double ps)
{
    if (kase != OR_NORMAL) return 0.0;
    double mx = 0.0;
    const double *K[2] = {L, R};
    for (int s = 0; s < 2; s++) {
        double m2 = sqrt((g + 1.0) / (2.0 * g) * ps / K[s][2] + (g - 1.0) / (2.0 * g));
        if (m2 > mx) mx = m2;
    }
    return mx;
}

void oracle_face_fluxes(const om_mesh *M, const om_params *prm, double dt,
                        const double *W, const double *grad, double *face_flux,
                        int32_t *fallback, int32_t *kase)
{
    oracle_face_fluxes_ex(M, prm, dt, W, grad, face_flux, fallback, kase, NULL, NULL);
}

void oracle_face_fluxes_ex(const om_mesh *M, const om_params *prm, double dt,
                           const double *W, const double *grad, double *face_flux,
                           int32_t *fallback, int32_t *kase, double *s_flux, double *mach)
{
    oracle_face_fluxes_full(M, prm, dt, NULL, W, grad, face_flux, fallback, kase, s_flux, mach);
}

/* With an external static gravitational field (Section 5.2, the standard */
/* coupling, applied to a field given per cell): accel [D][N] holds        */
/* g_i = -grad Phi at each cell, and the half-step prediction of each      */
/* side's velocity gains (dt/2) g_K. Reading: the kick belongs to the      */
/* extrapolated prediction, so a face that falls back to unextrapolated    */
/* states (non-positive prediction) takes none. accel NULL: no field.      */
/* One face f: the sides are predicted over pdt[s]/2 (each side's own
 * prediction interval; pdt[s] = dt in a global step) and the flux is
 * integrated over fdt: out[c] = fdt A_f Fhat_c. wf holds the face
 * velocities. Returns the positivity fallback flag; the Riemann case, the
 * entropy flux and the Mach number go to the pointers that are set. */
static int face_flux_one(const om_mesh *M, const om_params *prm, const double *wf, int64_t f,
                         const double pdt[2], double fdt, const double *accel, const double *W,
                         const double *grad, double *out_flux, int32_t *kase_out, double *sflux_out,
                         double *mach_out)
{
    const int D = M->dim, nv = D + 2;
    const int64_t n = M->n_cells, nf = M->n_faces;
    const double g = prm->gamma;
    int64_t cell[2] = {M->face_L[f], M->face_R[f]};
    double d[3] = {0, 0, 0}, w[3] = {0, 0, 0}, nrm[3] = {0, 0, 0}, ell = 0.0;
    for (int k = 0; k < D; k++) { d[k] = M->face_sep[k * nf + f]; ell += d[k] * d[k]; w[k] = wf[k * nf + f]; }
    ell = sqrt(ell);
    for (int k = 0; k < D; k++) nrm[k] = d[k] / ell;

    double Wp[2][5], Wpp[2][5];
    for (int s = 0; s < 2; s++) {
        int64_t i = cell[s];
        double dx[3] = {0, 0, 0}, gr[5][3];
        for (int k = 0; k < D; k++)
            dx[k] = M->face_ctr[k * nf + f] - (s ? d[k] : 0.0) - M->centroid_off[k * n + i];
        Wp[s][0] = W[0 * n + i];
        for (int k = 0; k < D; k++) Wp[s][1 + k] = W[(1 + k) * n + i] - w[k];
        Wp[s][nv - 1] = W[(nv - 1) * n + i];
        for (int c = 0; c < nv; c++)
            for (int k = 0; k < D; k++) gr[c][k] = grad[(c * D + k) * n + i];
        half_step(D, g, pdt[s], Wp[s], gr, dx, Wpp[s]);
        if (accel)
            for (int k = 0; k < D; k++) Wpp[s][1 + k] += 0.5 * pdt[s] * accel[k * n + i];
    }
    int fb = !(Wpp[0][0] > 0.0 && Wpp[0][nv - 1] > 0.0 && Wpp[1][0] > 0.0 && Wpp[1][nv - 1] > 0.0);
    if (fb) memcpy(Wpp, Wp, sizeof(Wp));

    /* normal / transverse split */
    double un[2], tr[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (int s = 0; s < 2; s++) {
        double u = 0.0;
        for (int k = 0; k < D; k++) u += Wpp[s][1 + k] * nrm[k];
        un[s] = u;
        for (int k = 0; k < D; k++) tr[s][k] = Wpp[s][1 + k] - u * nrm[k];
    }
    double Ls[3] = {Wpp[0][0], un[0], Wpp[0][nv - 1]};
    double Rs[3] = {Wpp[1][0], un[1], Wpp[1][nv - 1]};
    double out[4], st[2];
    int k0 = oracle_riemann(g, Ls, Rs, out, st, NULL);
    if (kase_out) *kase_out = k0;
    double rhoF = out[0], uF = out[1], PF = out[2];
    int side = out[3] > 0.5;

    double vF[3] = {0, 0, 0};
    for (int k = 0; k < D; k++) vF[k] = uF * nrm[k] + tr[side][k];
    double mf = rhoF * uF;
    double v2 = 0.0, w2 = 0.0, Piw = 0.0, Pi[3] = {0, 0, 0};
    for (int k = 0; k < D; k++) {
        v2 += vF[k] * vF[k];
        w2 += w[k] * w[k];
        Pi[k] = mf * vF[k] + PF * nrm[k];
        Piw += Pi[k] * w[k];
    }
    double eps = mf * 0.5 * v2 + uF * PF * g / (g - 1.0);
    double scale = fdt * M->face_area[f];
    out_flux[0] = scale * mf;
    for (int k = 0; k < D; k++) out_flux[1 + k] = scale * (Pi[k] + mf * w[k]);
    out_flux[nv - 1] = scale * (eps + Piw + 0.5 * mf * w2);
    if (sflux_out) {
        const double *U = side ? Rs : Ls;
        *sflux_out = (mf != 0.0) ? scale * mf * (U[2] / pow(U[0], g)) : 0.0;
    }
    if (mach_out) *mach_out = riemann_shock_mach(g, Ls, Rs, k0, st[0]);
    return fb;
}

void oracle_face_fluxes_full(const om_mesh *M, const om_params *prm, double dt, const double *accel,
                             const double *W, const double *grad, double *face_flux,
                             int32_t *fallback, int32_t *kase, double *s_flux, double *mach)
{
    const int nv = M->dim + 2;
    const int64_t nf = M->n_faces;
    const double pdt[2] = {dt, dt};
    double *wf = (double *)malloc(sizeof(double) * M->dim * nf);
    oracle_face_velocity(M, wf);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t f = 0; f < nf; f++) {
        double F[5];
        int fb = face_flux_one(M, prm, wf, f, pdt, dt, accel, W, grad, F, kase ? kase + f : NULL,
                               s_flux ? s_flux + f : NULL, mach ? mach + f : NULL);
        if (fallback) fallback[f] = fb;
        for (int c = 0; c < nv; c++) face_flux[c * nf + f] = F[c];
    }
    free(wf);
}

/* ------------------------------------------------------------------ */
/* Step (vii): conservative update, Q_i <- Q_i - dt sum_j A_ij F_ij,     */
/* with F_ji = -F_ij (Section 3, discrete update): the left cell loses   */
/* the face flux and the right cell gains it, in face-list order.        */
/* ------------------------------------------------------------------ */
static void apply_update_with(const om_mesh *M, const om_sides *S, const double *face_flux, double *Q)
{
    const int nv = M->dim + 2;
    const int64_t n = M->n_cells, nf = M->n_faces;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++)
        for (int64_t q = S->off[i]; q < S->off[i + 1]; q++) {
            const int64_t f = S->face[q];
            for (int c = 0; c < nv; c++) {
                if (S->right[q]) Q[c * n + i] += face_flux[c * nf + f];
                else Q[c * n + i] -= face_flux[c * nf + f];
            }
        }
}

void oracle_apply_update(const om_mesh *M, const double *face_flux, double *Q)
{
    om_sides S;
    sides_build(M, &S);
    apply_update_with(M, &S, face_flux, Q);
    sides_free(&S);
}

/* ------------------------------------------------------------------ */
/* Step (v): global Courant timestep (Section 7.1):                      */
/*   dt = C min_i R_i / (c_i + |v_i - w_i|),                             */
/* R_i = (3V/4pi)^(1/3) in 3D, (V/pi)^(1/2) in 2D. Vacuum cells (rho<=0  */
/* or P<=0) impose no limit.                                             */
/* ------------------------------------------------------------------ */
double oracle_cfl_dt(const om_mesh *M, const om_params *prm, const double *W)
{
    const int D = M->dim, nv = D + 2;
    const int64_t n = M->n_cells;
    double best = INFINITY;
    /* per-thread minima, then their minimum (a minimum is exact in any order) */
#pragma omp parallel
    {
    double mine = INFINITY;
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double rho = W[0 * n + i], P = W[(nv - 1) * n + i];
        if (!(rho > 0.0 && P > 0.0)) continue;
        double R = (D == 3) ? cbrt(3.0 * M->volume[i] / (4.0 * PI_D)) : sqrt(M->volume[i] / PI_D);
        double c = sqrt(prm->gamma * P / rho);
        double rel = 0.0;
        for (int k = 0; k < D; k++) {
            double dv = W[(1 + k) * n + i] - M->mesh_vel[k * n + i];
            rel += dv * dv;
        }
        double dti = prm->cfl * R / (c + sqrt(rel));
        if (dti < mine) mine = dti;
    }
#pragma omp critical
    if (mine < best) best = mine;
    }
    return best;
}

/* ------------------------------------------------------------------ */
/* Steps (ii), (iii), (v), (vi), (vii) in the order of Section 3's step  */
/* list. dt <= 0 requests the Courant timestep. Q is updated in place.   */
/* Returns the timestep used.                                            */
/* ------------------------------------------------------------------ */
double oracle_hydro_step(const om_mesh *M, const om_params *prm, double dt, double *Q)
{
    const int D = M->dim, nv = D + 2;
    const int64_t n = M->n_cells, nf = M->n_faces;
    double *W = (double *)malloc(sizeof(double) * nv * n);
    double *gr = (double *)malloc(sizeof(double) * nv * D * n);
    double *gl = (double *)malloc(sizeof(double) * nv * D * n);
    double *fl = (double *)malloc(sizeof(double) * nv * nf);
    om_sides S;
    sides_build(M, &S);
    oracle_prim(D, n, prm->gamma, M->volume, Q, W);
    gradients_with(M, &S, W, gr, gl, NULL);
    if (!(dt > 0.0)) dt = oracle_cfl_dt(M, prm, W);
    oracle_face_fluxes(M, prm, dt, W, gl, fl, NULL, NULL);
    apply_update_with(M, &S, fl, Q);
    sides_free(&S);
    free(W); free(gr); free(gl); free(fl);
    return dt;
}

/* ------------------------------------------------------------------ */
/* Section 3.5: the total entropy S_i = M_i A_i, A = P / rho^g, carried  */
/* as one more conserved row of Q ([D+3][N], S last) and advected by the */
/* entropy fluxes. After the conservative update of all rows, a cell     */
/* whose surrounding Riemann problems hold no shock of Mach number       */
/* mach_thresh or more keeps its advected entropy: its pressure follows  */
/* from it, P = (S/M) rho^g, and its total energy is rebuilt as          */
/* P V/(g-1) + |p|^2/(2M). Every other cell discards the advected value  */
/* and takes S = M P / rho^g of its updated state. Reading: a cell keeps */
/* only with positive new mass and entropy; mach_thresh <= 0 never keeps.*/
/* kept [N] (may be NULL) receives 1 where the entropy was kept.         */
/* ------------------------------------------------------------------ */
void oracle_update_full(const om_mesh *M, const om_params *prm, double dt, const double *accel,
                        const double *face_flux, const double *s_flux, const double *mach, double mach_thresh,
                        double *Q, int32_t *kept);

void oracle_apply_update_entropy(const om_mesh *M, const om_params *prm, const double *face_flux,
                                 const double *s_flux, const double *mach, double mach_thresh,
                                 double *Q, int32_t *kept)
{
    oracle_update_full(M, prm, 0.0, NULL, face_flux, s_flux, mach, mach_thresh, Q, kept);
}

/* The update with the optional parts: after the conservative sums of all */
/* rows, the gravitational source terms of Section 5.2 for a static field */
/* g_i (accel, may be NULL), with m_i^(n+1) from the mass fluxes:          */
/*   p_i += (dt/2) (m_i^(n) + m_i^(n+1)) g_i,                              */
/*   E_i += (dt/2) (p_i^(n) + p_i^(n+1)) . g_i  (m v at both ends),        */
/* then, with s_flux (may be NULL), the entropy treatment above.          */
/* The keep decision of the entropy treatment: with mode 1 the Mach number */
/* switch above; with mode 2 the energy switch of Section 3.5 (eqs.       */
/* eqnScrit1, eqnScrit2): a cell is cold and keeps its advected entropy   */
/* when its expected new thermal energy E_th = E - M v^2/2 (after the      */
/* conservative update and the gravitational sources) satisfies            */
/*   alpha_s > 0 and E_th < alpha_s E_kin^max,  or                         */
/*   beta_s > 0, a field given, and E_th < beta_s M |g_i| R_i,             */
/* with E_kin^max the largest M_j |v_j - w_i|^2 / 2 over the cell and its   */
/* face neighbours, measured in the frame of the cell's generator (w_i)    */
/* from the states at the start of the step (the neighbours' new states    */
/* are not known while the cell is updated), and R_i the radius of the     */
/* cell's volume. Readings: the start-of-step states; alpha_s or beta_s    */
/* <= 0 switches its condition off; M in eqnScrit2 is the new mass.       */
typedef struct {
    int mode;               /* 1 Mach number, 2 energy */
    double mach_thresh, alpha_s, beta_s;
} om_switch;

static void update_core(const om_mesh *M, const om_params *prm, double dt, const double *accel,
                        const double *face_flux, const double *s_flux, const double *mach, const om_switch *sw,
                        double *Q, int32_t *kept);

void oracle_update_full(const om_mesh *M, const om_params *prm, double dt, const double *accel,
                        const double *face_flux, const double *s_flux, const double *mach, double mach_thresh,
                        double *Q, int32_t *kept)
{
    const om_switch sw = {1, mach_thresh, 0.0, 0.0};
    update_core(M, prm, dt, accel, face_flux, s_flux, mach, &sw, Q, kept);
}

void oracle_update_energy_switch(const om_mesh *M, const om_params *prm, double dt, const double *accel,
                                 const double *face_flux, const double *s_flux, double alpha_s, double beta_s,
                                 double *Q, int32_t *kept)
{
    const om_switch sw = {2, 0.0, alpha_s, beta_s};
    update_core(M, prm, dt, accel, face_flux, s_flux, NULL, &sw, Q, kept);
}

static void update_core(const om_mesh *M, const om_params *prm, double dt, const double *accel,
                        const double *face_flux, const double *s_flux, const double *mach, const om_switch *sw,
                        double *Q, int32_t *kept)
{
    const int D = M->dim, nv = D + 2;
    const int64_t n = M->n_cells, nf = M->n_faces;
    const double g = prm->gamma;
    double *old = NULL, *ekmax = NULL;
    if (accel) {
        old = (double *)malloc(sizeof(double) * (D + 1) * n);
        memcpy(old, Q, sizeof(double) * (D + 1) * n);        /* m, p at the start */
    }
    if (s_flux && sw->mode == 2) {
        /* E_kin^max from the start-of-step states, in each cell's frame */
        ekmax = (double *)malloc(sizeof(double) * n);
        double *vel = (double *)calloc((size_t)D * n, sizeof(double));
        for (int64_t i = 0; i < n; i++)
            if (Q[i] > 0.0)
                for (int k = 0; k < D; k++) vel[k * n + i] = Q[(1 + k) * n + i] / Q[i];
        for (int64_t i = 0; i < n; i++) {
            double e = 0.0;
            for (int k = 0; k < D; k++) {
                const double dv = vel[k * n + i] - M->mesh_vel[k * n + i];
                e += dv * dv;
            }
            ekmax[i] = Q[i] > 0.0 ? 0.5 * Q[i] * e : 0.0;
        }
        for (int64_t f = 0; f < nf; f++) {
            const int64_t cell[2] = {M->face_L[f], M->face_R[f]};
            for (int s2 = 0; s2 < 2; s2++) {
                const int64_t i = cell[s2], j = cell[1 - s2];
                if (!(Q[j] > 0.0)) continue;
                double e = 0.0;
                for (int k = 0; k < D; k++) {
                    const double dv = vel[k * n + j] - M->mesh_vel[k * n + i];
                    e += dv * dv;
                }
                e *= 0.5 * Q[j];
                if (e > ekmax[i]) ekmax[i] = e;
            }
        }
        free(vel);
    }
    oracle_apply_update(M, face_flux, Q);
    if (accel) {
        for (int64_t i = 0; i < n; i++) {
            const double m0 = old[i], m1 = Q[i];
            double work = 0.0;
            for (int k = 0; k < D; k++) {
                const double gk = accel[k * n + i], p0 = old[(1 + k) * n + i];
                const double p1 = Q[(1 + k) * n + i] + 0.5 * dt * (m0 + m1) * gk;
                Q[(1 + k) * n + i] = p1;
                work += (p0 + p1) * gk;
            }
            Q[(nv - 1) * n + i] += 0.5 * dt * work;
        }
        free(old);
    }
    if (!s_flux) return;
    double *mmax = (double *)calloc((size_t)n, sizeof(double));
    for (int64_t f = 0; f < nf; f++) {
        int64_t l = M->face_L[f], r = M->face_R[f];
        Q[nv * n + l] -= s_flux[f];
        Q[nv * n + r] += s_flux[f];
        if (mach) {
            if (mach[f] > mmax[l]) mmax[l] = mach[f];
            if (mach[f] > mmax[r]) mmax[r] = mach[f];
        }
    }
    for (int64_t i = 0; i < n; i++) {
        const double m = Q[i], V = M->volume[i], S = Q[nv * n + i];
        double p2 = 0.0;
        for (int k = 0; k < D; k++) p2 += Q[(1 + k) * n + i] * Q[(1 + k) * n + i];
        int cold;
        if (sw->mode == 1) {
            cold = mmax[i] < sw->mach_thresh;
        } else {
            const double eth = m > 0.0 ? Q[(nv - 1) * n + i] - 0.5 * p2 / m : 0.0;
            cold = sw->alpha_s > 0.0 && eth < sw->alpha_s * ekmax[i];
            if (!cold && sw->beta_s > 0.0 && accel) {
                double g2 = 0.0;
                for (int k = 0; k < D; k++) g2 += accel[k * n + i] * accel[k * n + i];
                const double R = (D == 3) ? cbrt(3.0 * V / (4.0 * PI_D)) : sqrt(V / PI_D);
                cold = eth < sw->beta_s * m * sqrt(g2) * R;
            }
        }
        const int keep = cold && m > 0.0 && S > 0.0;
        if (kept) kept[i] = keep;
        if (!(m > 0.0)) { Q[nv * n + i] = 0.0; continue; }
        const double rho = m / V, ke = 0.5 * p2 / m;
        if (keep) {
            const double P = (S / m) * pow(rho, g);
            Q[(nv - 1) * n + i] = P * V / (g - 1.0) + ke;
        } else {
            const double P = (g - 1.0) * (Q[(nv - 1) * n + i] - ke) / V;
            Q[nv * n + i] = m * P / pow(rho, g);
        }
    }
    free(mmax);
    free(ekmax);
}

/* The step with the entropy row: primitives, gradients, timestep and     */
/* face states exactly as oracle_hydro_step (from the first D+2 rows),   */
/* then the entropy update above.                                        */
double oracle_hydro_step_entropy(const om_mesh *M, const om_params *prm, double dt, double mach_thresh,
                                 double *Q, int32_t *kept)
{
    const int D = M->dim, nv = D + 2;
    const int64_t n = M->n_cells, nf = M->n_faces;
    double *W = (double *)malloc(sizeof(double) * nv * n);
    double *gr = (double *)malloc(sizeof(double) * nv * D * n);
    double *gl = (double *)malloc(sizeof(double) * nv * D * n);
    double *fl = (double *)malloc(sizeof(double) * nv * nf);
    double *sf = (double *)malloc(sizeof(double) * nf);
    double *mc = (double *)malloc(sizeof(double) * nf);
    oracle_prim(D, n, prm->gamma, M->volume, Q, W);
    oracle_gradients(M, W, gr, gl, NULL);
    if (!(dt > 0.0)) dt = oracle_cfl_dt(M, prm, W);
    oracle_face_fluxes_ex(M, prm, dt, W, gl, fl, NULL, NULL, sf, mc);
    oracle_apply_update_entropy(M, prm, fl, sf, mc, mach_thresh, Q, kept);
    free(W); free(gr); free(gl); free(fl); free(sf); free(mc);
    return dt;
}

/* The largest shock Mach number of one Riemann problem (the face rule    */
/* above), with its star pressure; for tests.                            */
double oracle_shock_mach(double g, const double *L, const double *R)
{
    double out[4], st[2];
    int k = oracle_riemann(g, L, R, out, st, NULL);
    return riemann_shock_mach(g, L, R, k, st[0]);
}

/* ------------------------------------------------------------------ */
/* Mesh motion (Section 3.2 and Section 4.1). The generators move with   */
/* their cell's fluid velocity, w_i = v_i (eq. eqnvelmesh), plus the     */
/* roundness correction of eq. EqnShapeCorrVel: with d_i = |s_i - r_i|,  */
/* R_i = (3 V_i / 4 pi)^(1/3) in 3D ((V_i / pi)^(1/2) in 2D) and         */
/* x = d_i / (eta R_i), add chi times                                    */
/*   0                                            for x < 0.9            */
/*   c_i (s_i - r_i)/d_i (d_i - 0.9 eta R_i)/(0.2 eta R_i)  0.9 <= x < 1.1*/
/*   c_i (s_i - r_i)/d_i                          for 1.1 <= x           */
/* with c_i the cell's sound speed, or, when dt_lloyd > 0, the paper's   */
/* alternative (s_i - r_i)/dt_lloyd in place of c_i (s_i - r_i)/d_i.     */
/* W are primitives; a vacuum cell (rho <= 0 or P <= 0) has c_i = 0.     */
/* w_out [D][N].                                                         */
/* ------------------------------------------------------------------ */
void oracle_mesh_velocity(const om_mesh *M, const om_params *prm, const double *W, double eta, double chi,
                          double dt_lloyd, double *w_out)
{
    const int D = M->dim;
    const int64_t n = M->n_cells;
    for (int64_t i = 0; i < n; i++) {
        double sr[3] = {0, 0, 0}, d = 0.0;
        for (int k = 0; k < D; k++) { sr[k] = M->centroid_off[k * n + i]; d += sr[k] * sr[k]; }
        d = sqrt(d);
        const double V = M->volume[i];
        const double R = (D == 3) ? cbrt(3.0 * V / (4.0 * PI_D)) : sqrt(V / PI_D);
        const double rho = W[i], P = W[(D + 1) * n + i];
        const double c = (rho > 0.0 && P > 0.0) ? sqrt(prm->gamma * P / rho) : 0.0;
        const double x = d / (eta * R);
        double frac = 0.0;
        if (x >= 1.1) frac = 1.0;
        else if (x >= 0.9) frac = (d - 0.9 * eta * R) / (0.2 * eta * R);
        for (int k = 0; k < D; k++) {
            double corr = 0.0;
            if (frac > 0.0) corr = (dt_lloyd > 0.0) ? sr[k] / dt_lloyd : c * sr[k] / d;
            w_out[k * n + i] = W[(1 + k) * n + i] + chi * frac * corr;
        }
    }
}

/* Rate of change of each cell's volume from the generator velocities    */
/* (Section 3.3, eq. eqnvolchange), summed over the cell's faces as      */
/* printed: dV_i/dt = - sum_j A_ij [ c_ij/r_ij . (w_j - w_i)             */
/*                                   + r_ij/(2 r_ij) . (w_j + w_i) ],    */
/* r_ij = r_i - r_j (periodic image), c_ij = f_ij - (r_i + r_j)/2.       */
/* rate [N].                                                             */
void oracle_volume_rate(const om_mesh *M, double *rate)
{
    const int D = M->dim;
    const int64_t n = M->n_cells, nf = M->n_faces;
    for (int64_t i = 0; i < n; i++) rate[i] = 0.0;
    for (int64_t f = 0; f < nf; f++) {
        const int64_t cell[2] = {M->face_L[f], M->face_R[f]};
        double d[3] = {0, 0, 0}, cc[3] = {0, 0, 0}, len = 0.0;
        for (int k = 0; k < D; k++) {
            d[k] = M->face_sep[k * nf + f];                 /* r_R - r_L */
            cc[k] = M->face_ctr[k * nf + f] - 0.5 * d[k];   /* f - (r_L + r_R)/2 */
            len += d[k] * d[k];
        }
        len = sqrt(len);
        for (int s = 0; s < 2; s++) {
            const int64_t i = cell[s], j = cell[1 - s];
            double term = 0.0;
            for (int k = 0; k < D; k++) {
                const double rij = s == 0 ? -d[k] : d[k];      /* r_i - r_j */
                const double wi = M->mesh_vel[k * n + i], wj = M->mesh_vel[k * n + j];
                term += cc[k] / len * (wj - wi) + rij / (2.0 * len) * (wj + wi);
            }
            rate[i] -= M->face_area[f] * term;
        }
    }
}

/* The step with every option: static gravity (accel [D][N] or NULL) and */
/* the entropy row (entropy != 0: Q is [D+3][N]).                         */
double oracle_hydro_step_full(const om_mesh *M, const om_params *prm, double dt, const double *accel,
                              int entropy, double mach_thresh, double *Q, int32_t *kept)
{
    const int D = M->dim, nv = D + 2;
    const int64_t n = M->n_cells, nf = M->n_faces;
    double *W = (double *)malloc(sizeof(double) * nv * n);
    double *gr = (double *)malloc(sizeof(double) * nv * D * n);
    double *gl = (double *)malloc(sizeof(double) * nv * D * n);
    double *fl = (double *)malloc(sizeof(double) * nv * nf);
    double *sf = entropy ? (double *)malloc(sizeof(double) * nf) : NULL;
    double *mc = entropy ? (double *)malloc(sizeof(double) * nf) : NULL;
    oracle_prim(D, n, prm->gamma, M->volume, Q, W);
    oracle_gradients(M, W, gr, gl, NULL);
    if (!(dt > 0.0)) dt = oracle_cfl_dt(M, prm, W);
    oracle_face_fluxes_full(M, prm, dt, accel, W, gl, fl, NULL, NULL, sf, mc);
    oracle_update_full(M, prm, dt, accel, fl, sf, mc, mach_thresh, Q, kept);
    free(W); free(gr); free(gl); free(fl); free(sf); free(mc);
    return dt;
}

/* ------------------------------------------------------------------ */
/* Section 7.2, individual timesteps.                                    */
/*                                                                       */
/* Criterion (eq. EqnTiStepIndividual, with the minimum over j taken over */
/* the Voronoi neighbours only; the paper's tree walk over all cells is   */
/* not modelled):                                                        */
/*   dt_i = C min(tau_i, R_i / (c_i + |v_i - w_i|)),                     */
/*   tau_i = min_j r_ij / v_sig_ij,                                      */
/*   v_sig_ij = c_i + c_j - (v_i - v_j).(r_i - r_j)/r_ij.                */
/* For a face with normal n = d/|d| (L to R) the projection is the same   */
/* from both sides, (v_i - v_j).(r_i - r_j)/r_ij = (v_R - v_L).n, so each */
/* face has one signal speed. Readings: a pair with v_sig <= 0 (receding */
/* faster than sound) sets no bound; a vacuum cell (rho <= 0 or P <= 0)   */
/* has c = 0 and sets no local bound, like the global Courant step.       */
/* dt_out [N].                                                           */
/* ------------------------------------------------------------------ */
void oracle_tb_criterion(const om_mesh *M, const om_params *prm, const double *W, double *dt_out)
{
    const int D = M->dim, nv = D + 2;
    const int64_t n = M->n_cells, nf = M->n_faces;
    double *c = (double *)malloc(sizeof(double) * n);
    double *tau = (double *)malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; i++) {
        const double rho = W[i], P = W[(nv - 1) * n + i];
        c[i] = (rho > 0.0 && P > 0.0) ? sqrt(prm->gamma * P / rho) : 0.0;
        tau[i] = INFINITY;
    }
    for (int64_t f = 0; f < nf; f++) {
        const int64_t l = M->face_L[f], r = M->face_R[f];
        double ell = 0.0, du = 0.0;
        for (int k = 0; k < D; k++) ell += M->face_sep[k * nf + f] * M->face_sep[k * nf + f];
        ell = sqrt(ell);
        for (int k = 0; k < D; k++)
            du += (W[(1 + k) * n + r] - W[(1 + k) * n + l]) * (M->face_sep[k * nf + f] / ell);
        const double vsig = (c[l] + c[r]) - du;
        if (vsig > 0.0) {
            const double t = ell / vsig;
            if (t < tau[l]) tau[l] = t;
            if (t < tau[r]) tau[r] = t;
        }
    }
    for (int64_t i = 0; i < n; i++) {
        const double rho = W[i], P = W[(nv - 1) * n + i];
        double loc = INFINITY;
        if (rho > 0.0 && P > 0.0) {
            const double V = M->volume[i];
            const double R = (D == 3) ? cbrt(3.0 * V / (4.0 * PI_D)) : sqrt(V / PI_D);
            double rel = 0.0;
            for (int k = 0; k < D; k++) {
                const double dv = W[(1 + k) * n + i] - M->mesh_vel[k * n + i];
                rel += dv * dv;
            }
            loc = R / (c[i] + sqrt(rel));
        }
        dt_out[i] = prm->cfl * (tau[i] < loc ? tau[i] : loc);
    }
    free(c);
    free(tau);
}

/* ------------------------------------------------------------------ */
/* One synchronisation point of the individual-timestep integration      */
/* (Section 7.2). Time is counted in ticks of dt_max / 2^L; a cell in bin */
/* b takes steps of 2^b ticks that start at multiples of 2^b (the power-  */
/* of-two hierarchy; bin L is the step dt_max). At tick ti:              */
/*  1. the cells whose step ends now (ti a multiple of 2^bin) are active: */
/*     their primitives are recomputed from Q and stamped trec = ti;      */
/*  2. each active cell takes the bin of the largest power-of-two         */
/*     subdivision of dt_max not above its criterion dt_i; it may move    */
/*     down any number of bins, but up by one bin only, and only when the */
/*     higher bin starts a step at ti (at most every second step);        */
/*  3. the gradients (with the limiter) of the active cells are rebuilt   */
/*     from the stored primitives of all cells: fresh for the active,     */
/*     those of the last active step for the rest;                       */
/*  4. a face is active when the smaller step of its two cells starts at  */
/*     ti; it is integrated over that step, fdt = 2^min(bL,bR) ticks, and */
/*     each side is predicted from its stored record to the middle of the */
/*     face's step, (ti - trec) ticks + fdt/2 after the record was made;  */
/*     both cells exchange the time-integrated flux (conservative);       */
/*  5. the next synchronisation point is the next multiple of the step of */
/*     the smallest occupied bin.                                        */
/* Arrays carried between calls: bin [N] (int8; all L before the first   */
/* call, when every cell is due), trec [N], W [D+2][N], G [(D+2)D][N].   */
/* face_dt [F] (may be NULL) receives fdt of the active faces, 0 for the  */
/* others; pred [2][F] (may be NULL) the prediction interval of each side */
/* (left, right) of the active faces; active [N] (may be NULL) 1 for the  */
/* active cells. Returns 0, or                                           */
/* 1 when an active cell's criterion falls below one tick (no bin fits):  */
/* then steps 3-5 are not done and Q is untouched.                       */
/* ------------------------------------------------------------------ */
int oracle_tb_step(const om_mesh *M, const om_params *prm, double dt_max, int32_t L, int64_t ti,
                   int8_t *bin, int64_t *trec, double *W, double *G, double *Q, double *face_dt,
                   double *pred, int32_t *active, int64_t *next_ti, int64_t *n_active_faces)
{
    const int D = M->dim, nv = D + 2;
    const int64_t n = M->n_cells, nf = M->n_faces;
    const double tick = ldexp(dt_max, -L);
    int8_t *act = (int8_t *)malloc(n);
    double *Wn = (double *)malloc(sizeof(double) * nv * n);
    double *dti = (double *)malloc(sizeof(double) * n);
    int status = 0;

    /* 1 */
    oracle_prim(D, n, prm->gamma, M->volume, Q, Wn);
    for (int64_t i = 0; i < n; i++) {
        act[i] = (ti & ((INT64_C(1) << bin[i]) - 1)) == 0;
        if (active) active[i] = act[i];
        if (!act[i]) continue;
        trec[i] = ti;
        for (int c = 0; c < nv; c++) W[c * n + i] = Wn[c * n + i];
    }
    /* 2 */
    oracle_tb_criterion(M, prm, W, dti);
    for (int64_t i = 0; i < n; i++) {
        if (!act[i]) continue;
        if (!(dti[i] >= tick)) { status = 1; continue; }
        int b = L;
        while (b > 0 && ldexp(dt_max, b - L) > dti[i]) b--;
        const int old = bin[i];
        if (b <= old) bin[i] = (int8_t)b;
        else if ((ti & ((INT64_C(1) << (old + 1)) - 1)) == 0) bin[i] = (int8_t)(old + 1);
    }
    if (status) goto done;
    /* 3 */
    {
        double *gr = (double *)malloc(sizeof(double) * nv * D * n);
        double *gl = (double *)malloc(sizeof(double) * nv * D * n);
        oracle_gradients(M, W, gr, gl, NULL);
        for (int64_t i = 0; i < n; i++)
            if (act[i])
                for (int c = 0; c < nv * D; c++) G[c * n + i] = gl[c * n + i];
        free(gr);
        free(gl);
    }
    /* 4 */
    {
        double *wf = (double *)malloc(sizeof(double) * D * nf);
        oracle_face_velocity(M, wf);
        int64_t na = 0;
        for (int64_t f = 0; f < nf; f++) {
            const int64_t cell[2] = {M->face_L[f], M->face_R[f]};
            const int b = bin[cell[0]] < bin[cell[1]] ? bin[cell[0]] : bin[cell[1]];
            if (face_dt) face_dt[f] = 0.0;
            if (pred) { pred[f] = 0.0; pred[nf + f] = 0.0; }
            if ((ti & ((INT64_C(1) << b) - 1)) != 0) continue;
            const double fdt = ldexp(dt_max, b - L);
            double pdt[2];
            for (int s = 0; s < 2; s++) pdt[s] = 2.0 * ((double)(ti - trec[cell[s]]) * tick + 0.5 * fdt);
            double F[5];
            face_flux_one(M, prm, wf, f, pdt, fdt, NULL, W, G, F, NULL, NULL, NULL);
            for (int c = 0; c < nv; c++) {
                Q[c * n + cell[0]] -= F[c];
                Q[c * n + cell[1]] += F[c];
            }
            if (face_dt) face_dt[f] = fdt;
            if (pred) { pred[f] = 0.5 * pdt[0]; pred[nf + f] = 0.5 * pdt[1]; }
            na++;
        }
        if (n_active_faces) *n_active_faces = na;
        free(wf);
    }
    /* 5 */
    {
        int b0 = L;
        for (int64_t i = 0; i < n; i++)
            if (bin[i] < b0) b0 = bin[i];
        if (next_ti) *next_ti = ((ti >> b0) + 1) << b0;
    }
done:
    free(act);
    free(Wn);
    free(dti);
    return status;
}

/* The step with the energy switch of the entropy treatment (Section 3.5, */
/* eqs. eqnScrit1-eqnScrit2) and an optional static field: as             */
/* oracle_hydro_step_full with update_core's mode 2.                     */
double oracle_hydro_step_energy(const om_mesh *M, const om_params *prm, double dt, const double *accel,
                                double alpha_s, double beta_s, double *Q, int32_t *kept)
{
    const int D = M->dim, nv = D + 2;
    const int64_t n = M->n_cells, nf = M->n_faces;
    double *W = (double *)malloc(sizeof(double) * nv * n);
    double *gr = (double *)malloc(sizeof(double) * nv * D * n);
    double *gl = (double *)malloc(sizeof(double) * nv * D * n);
    double *fl = (double *)malloc(sizeof(double) * nv * nf);
    double *sf = (double *)malloc(sizeof(double) * nf);
    oracle_prim(D, n, prm->gamma, M->volume, Q, W);
    oracle_gradients(M, W, gr, gl, NULL);
    if (!(dt > 0.0)) dt = oracle_cfl_dt(M, prm, W);
    oracle_face_fluxes_full(M, prm, dt, accel, W, gl, fl, NULL, NULL, sf, NULL);
    oracle_update_energy_switch(M, prm, dt, accel, fl, sf, alpha_s, beta_s, Q, kept);
    free(W); free(gr); free(gl); free(fl); free(sf);
    return dt;
}

/* ------------------------------------------------------------------ */
/* Reflective walls by mirrored generators (Section 3.6, boundary     */
/* conditions): each ghost cell g takes the                           */
/* conserved state of its source cell with the momentum component     */
/* normal to the wall (row 1 + axis) negated, all nrow rows of Q      */
/* [nrow][N] (the entropy row included when present). The ghosts'      */
/* generators are the sources' mirror images, so the wall face between */
/* a cell and its image carries a symmetric Riemann problem: no mass   */
/* or energy flux, and the momentum flux of the star pressure; the     */
/* reflective condition for the moving-mesh scheme.                   */
/* ------------------------------------------------------------------ */
void oracle_reflect(int32_t nrow, int64_t n, double *Q, int64_t n_ghost, const int32_t *ghost,
                    const int32_t *src, int32_t axis)
{
    for (int64_t k = 0; k < n_ghost; k++) {
        const int64_t g = ghost[k], s = src[k];
        for (int c = 0; c < nrow; c++) Q[c * n + g] = Q[c * n + s];
        Q[(1 + axis) * n + g] = -Q[(1 + axis) * n + s];
    }
}
