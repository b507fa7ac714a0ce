/*
 * mm.h -- C ABI of libmm: one second-order finite-volume hydro step of the
 * moving Voronoi-mesh Godunov scheme (Springel, "E pur si muove",
 * arXiv:0901.4107, Section 3) on a given periodic tessellation, on one
 * AMD Instinct MI355X (gfx950) GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller (for
 *   example the data pointer of a contiguous torch tensor). The library never
 *   allocates device memory: its scratch space is the workspace the caller
 *   hands over with mm_set_workspace.
 * - Conserved states Q are double, structure-of-arrays [D+2][N] (rows m,
 *   p_x, p_y(, p_z), E: cell totals); D is the dimension (2 or 3), N the
 *   number of cells, F the number of faces. With MM_ENTROPY_MACH, Q is
 *   [D+3][N], the total entropy S as last row.
 * - Face fluxes are double, face-major: face_flux[f*FS + c] =
 *   dt * A_f * Fhat_c(f), c over (mass, momentum (D), energy), FS =
 *   MM_FLUX_STRIDE(D, entropy) (with the entropy row, then the entropy
 *   flux, and with MM_ENTROPY_MACH the face's shock Mach number).
 * - The reconstruction buffer (mm_gradients' output) holds
 *   MM_RECON_STRIDE(D) elements per cell (24 in 3D, 16 in 2D) as two
 *   blocks:
 *     primitive block P [N][8]:  rho, v (D), P, s_i - r_i (D) (centre of mass
 *                                minus generator), padding
 *     gradient block  G [N][16] (3D) / [N][8] (2D), starting at element 8N:
 *                                limited gradient, element c*D + k =
 *                                dW_c/dx_k, padding
 *   In MM_FP64 its elements are double and v is the lab-frame velocity; in
 *   MM_MIXED they are float and v holds v_i - W0, W0 the midrange (min +
 *   max)/2 of the generator velocities per component at the last
 *   mm_mesh_upload or mm_mesh_set_velocity (the buffer belongs to that
 *   mesh state).
 * - The normal of face f points from its left cell face_L[f] to its right
 *   cell face_R[f]; Fhat(f) is the flux leaving the left cell.
 * - Calls enqueue work on params.stream (a hipStream_t; NULL = the null
 *   stream) and return without waiting, except where a call says it
 *   synchronises.
 * - Every call returns an mm_status and never throws. Numeric events inside
 *   a step (vacuum faces, positivity fallbacks, unconverged Newton
 *   iterations) are counted in the diagnostics, not returned as errors.
 * - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef MM_H
#define MM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mm_status;
#define MM_OK            0
#define MM_E_ARG        -1  /* null pointer, bad size, bad mode or dimension */
#define MM_E_MESH       -2  /* mesh validation failed (see mm_mesh_upload) */
#define MM_E_DEVICE     -3  /* a HIP runtime call failed */
#define MM_E_STATE      -4  /* call out of order: no workspace or no mesh */
#define MM_E_WORKSPACE  -5  /* workspace smaller than mm_workspace_bytes */
#define MM_E_NONFINITE  -6  /* a conserved quantity became NaN or infinite */
#define MM_E_RANGE      -7  /* a cell's timestep criterion is below the smallest
                               step of an individual-timestep timeline */

/* Arithmetic of the face-flux path. */
#define MM_FP64   0  /* every step in double precision */
#define MM_MIXED  1  /* single-precision reconstruction, frame transforms and
                        Riemann iterations on velocities relative to the
                        face; double-precision accumulation, lab-frame
                        transform, and Newton for hard faces */

/* Entropy treatment for poorly resolved cold flows (Section 3.5). With
 * MM_ENTROPY_MACH, Q carries the total entropy S_i = M_i P_i / rho_i^gamma
 * as one more row ([D+3][N], S last), advected by the entropy flux
 * m_F A_U of every face (A_U = P / rho^gamma of the upwind side of the
 * face's Riemann problem). After the update, a cell whose faces' Riemann
 * solutions hold no shock of Mach number mach_thresh or more (and whose new
 * mass and entropy are positive) keeps the advected entropy: its pressure
 * becomes (S/M) rho^gamma and its total energy P V/(gamma-1) + |p|^2/(2M),
 * so total energy is then not conserved. Every other cell takes
 * S = M P / rho^gamma of its conservatively updated state. */
#define MM_ENTROPY_OFF  0
#define MM_ENTROPY_MACH 1
/* The energy switch of the same section (eqs. eqnScrit1, eqnScrit2) in
 * place of the Mach number: a cell is cold, and keeps its entropy, when its
 * new thermal energy E - |p|^2/(2M) is below alpha_s times the largest
 * kinetic energy M_j |v_j - w_i|^2 / 2 of the cell and its face neighbours
 * (states at the start of the step, in the frame of the cell's generator),
 * or, with a static field (mm_set_gravity), below beta_s M |g_i| R_i, R_i
 * the radius of the cell's volume. A parameter <= 0 switches its condition
 * off. The gradient pass (mm_gradients, or the step's own) records each
 * cell's largest such energy (its own and its neighbours') in the
 * workspace, from the reconstruction records it takes the gradients of
 * (float in MM_MIXED); mm_apply_update returns MM_E_STATE before any
 * gradient pass. */
#define MM_ENTROPY_ENERGY 2

/* Timestep scheme (Section 7.2). MM_STEPS_INDIVIDUAL adds the arrays of a
 * power-of-two timeline to the workspace (mm_tb_begin, mm_tb_step); the
 * global step (mm_hydro_step) stays available. Not combined with the
 * entropy row. */
#define MM_STEPS_GLOBAL     0
#define MM_STEPS_INDIVIDUAL 1

/* Starting guess of the Newton iteration for the star pressure. */
#define MM_GUESS_STANDARD 0  /* adaptive PVRS / two-rarefaction / two-shock */
#define MM_GUESS_LEARNED  1  /* MLP loaded with mm_mlp_load */

typedef struct {
    int32_t dim;              /* 2 or 3 */
    int32_t mode;             /* MM_FP64 or MM_MIXED */
    int32_t guess;            /* MM_GUESS_STANDARD or MM_GUESS_LEARNED */
    int32_t newton_max_iter;  /* per face; <= 0 selects 50 */
    double gamma;             /* adiabatic index, > 1 */
    double cfl;               /* Courant factor of the timestep criterion */
    double newton_tol64;      /* relative Newton step tolerance, double; <= 0: 1e-10 */
    double newton_tol32;      /* same for the single-precision solve; <= 0: 1e-5 */
    void *stream;             /* hipStream_t */
    int32_t entropy;          /* MM_ENTROPY_OFF or MM_ENTROPY_MACH */
    int32_t steps;            /* MM_STEPS_GLOBAL or MM_STEPS_INDIVIDUAL */
    double mach_thresh;       /* MM_ENTROPY_MACH: cells whose largest face shock Mach
                                 number is below this keep their entropy (the paper
                                 suggests about 1.1); <= 0 never keeps; not NaN */
    double alpha_s;           /* MM_ENTROPY_ENERGY: eqnScrit1's factor (the paper uses
                                 about 0.01); >= 0 and finite */
    double beta_s;            /* MM_ENTROPY_ENERGY: eqnScrit2's factor; >= 0 and finite */
} mm_params;

/* Doubles per face record of the face-flux array: the D+2 fluxes
 * dt A Fhat, then with the entropy row the entropy flux dt A m_F A_U, and
 * with MM_ENTROPY_MACH (whose switch reads it; MM_ENTROPY_ENERGY's does
 * not, and its records end after the entropy flux) the face's Mach number:
 * the larger over its sides of
 * sqrt((g+1)/(2g) p* / p_K + (g-1)/(2g)), the Mach number of the shock into
 * side K where p* > p_K and below 1 on a rarefied side; 0 without a star
 * state. */
#define MM_FLUX_STRIDE(dim, entropy) \
    ((dim) + 2 + ((entropy) == MM_ENTROPY_MACH ? 2 : ((entropy) == MM_ENTROPY_ENERGY ? 1 : 0)))

/* The given tessellation (Section 3, step list item (i)) and the generator
 * velocities w_i (item (iv)). All device pointers, all kept by reference
 * until the next mm_mesh_upload or mm_destroy: the caller keeps them alive
 * and unchanged meanwhile. */
typedef struct {
    int64_t n_cells;             /* N >= 2 */
    int64_t n_faces;             /* F >= 1 */
    const double *volume;        /* [N]    V_i > 0 */
    const double *centroid_off;  /* [D][N] s_i - r_i (centre of mass minus generator) */
    const double *mesh_vel;      /* [D][N] generator velocities w_i */
    const int32_t *face_L;       /* [F]    0 <= L < N, non-decreasing in f (faces sorted by left cell) */
    const int32_t *face_R;       /* [F]    0 <= R < N, R != L */
    const double *face_area;     /* [F]    A_f >= 0 */
    const double *face_ctr;      /* [D][F] f - r_L, face centroid relative to L's generator */
    const double *face_sep;      /* [D][F] r_R - r_L, with R's periodic image; nonzero */
} mm_mesh;

typedef struct {
    uint64_t faces;              /* faces fluxed since the last reset */
    uint64_t newton_iters;       /* total Newton iterations */
    uint64_t newton_max;         /* largest iteration count of one face */
    uint64_t unconverged;        /* faces that hit newton_max_iter */
    uint64_t vacuum;             /* faces with a vacuum side or generated vacuum */
    uint64_t positivity_fallback;/* faces that used unextrapolated states */
    uint64_t fp64_fallback;      /* MM_MIXED: faces re-solved in double */
    uint64_t guess_fallback;     /* MM_GUESS_LEARNED: faces restarted from the standard guess */
    uint64_t wave_iter_max_sum;  /* sum over 64-lane wavefronts of their max iteration count,
                                    the wavefronts of the double re-solve pass included */
    uint64_t waves;              /* number of wavefronts of the main pass (faces or problems / 64) */
    uint64_t entropy_kept;       /* MM_ENTROPY_MACH: cell updates that kept the advected entropy */
    int32_t nonfinite;           /* 1 if a step produced a non-finite conserved value */
    int32_t reserved;
} mm_diag;

#define MM_RECON_STRIDE(dim) ((dim) == 3 ? 24 : 16)

typedef struct mm_ctx mm_ctx;

/* Create a context for the given parameters. Allocates host memory only.
 * MM_E_ARG for a bad dimension, mode, guess, entropy or steps value,
 * gamma <= 1, a NaN mach_thresh or a negative or non-finite alpha_s or
 * beta_s with their mode, or individual timesteps with the entropy row. */
mm_status mm_create(const mm_params *params, mm_ctx **out);

/* Destroy a context (NULL is accepted). Does not free the workspace. */
mm_status mm_destroy(mm_ctx *ctx);

/* Bytes of device workspace a mesh of n_cells cells and n_faces faces needs
 * for this context's dimension and mode; negative on bad arguments. */
int64_t mm_workspace_bytes(const mm_ctx *ctx, int64_t n_cells, int64_t n_faces);

/* Hand the context a device workspace (256-byte aligned) of `bytes` bytes.
 * The caller owns it and keeps it alive while the context uses it. */
mm_status mm_set_workspace(mm_ctx *ctx, void *dev_ptr, int64_t bytes);

/* Take a tessellation (Section 3, step (i)) and the generator velocities
 * (step (iv)). Validates it on the device, builds the per-cell list of faces
 * (in ascending face order), the face geometry and each face's velocity
 * (Section 3.3: the mean generator velocity plus the normal motion of the
 * face centroid induced by the generators' relative motion).
 * Synchronises the stream (to read the validation result).
 * MM_E_MESH if an index is out of range, L == R, a volume is not positive,
 * an area is negative, a separation is zero, any value is not finite, a
 * cell's faces do not close (|sum A n| > 1e-9 sum A; every Voronoi cell is
 * closed, and the gradient estimate relies on it), or the faces are not
 * sorted by left cell (face_L must not decrease: each cell's left faces are
 * then one contiguous range, which the face pass sums itself for the
 * update);
 * MM_E_WORKSPACE if the workspace is too small; MM_E_STATE without one. */
mm_status mm_mesh_upload(mm_ctx *ctx, const mm_mesh *mesh);

/* Steps (ii)-(iii): primitives W from Q (rho = m/V, v = p/m,
 * P = (gamma-1)(E - m v^2/2)/V; a cell with m <= 0 gets W = 0), then the
 * slope-limited gradients (Section 3.1: the Voronoi estimate exact to linear
 * order, limited per primitive so that face-centroid values stay within the
 * neighbourhood's extremes). Writes the reconstruction record of every cell
 * to `recon` (layout above; double in MM_FP64, float in MM_MIXED). */
mm_status mm_gradients(mm_ctx *ctx, const double *Q, void *recon);

/* Step (vi): the flux through every face over a step dt > 0 (Section 3.3:
 * extrapolation to the face centroid and half a step forward in time in the
 * face's rest frame, exact Riemann solution sampled on the face, moving-face
 * flux in the lab frame). `recon` as produced by mm_gradients in the same
 * mode. Writes face_flux [F][MM_FLUX_STRIDE] (double in every mode). */
mm_status mm_face_fluxes(mm_ctx *ctx, double dt, const void *recon, double *face_flux);

/* Step (vii): Q_L -= flux, Q_R += flux for every face (Section 3,
 * discrete update), summed per cell in a fixed order (bitwise reproducible);
 * face_flux [F][MM_FLUX_STRIDE] as written by mm_face_fluxes. With
 * MM_ENTROPY_MACH the entropy row is updated by its fluxes too and each
 * cell then keeps or re-derives its entropy as described at
 * MM_ENTROPY_MACH. */
mm_status mm_apply_update(mm_ctx *ctx, const double *face_flux, double *Q);

/* Steps (ii), (iii), (v), (vi), (vii) on Q in place. dt <= 0 selects the
 * global Courant timestep dt = C min_i R_i / (c_i + |v_i - w_i|) (Section
 * 7.1). If dt_used is non-NULL the call synchronises, stores the timestep
 * used there and returns MM_E_NONFINITE if this step left a non-finite
 * value in Q (the diagnostics' nonfinite flag keeps any such step until
 * mm_reset_diag); with dt_used NULL it returns without waiting. */
mm_status mm_hydro_step(mm_ctx *ctx, double *Q, double dt, double *dt_used);

/* MM_ENTROPY_MACH only (MM_E_ARG otherwise; MM_E_STATE without a mesh):
 * fill the entropy row of Q [D+3][N] from its other rows, S_i =
 * M_i P_i / rho_i^gamma with P from the total energy (Section 3.5's
 * definition; 0 where M_i <= 0). */
mm_status mm_entropy_init(mm_ctx *ctx, double *Q);

/* Mesh motion for the next tessellation (Section 3.2, eq. eqnvelmesh, and
 * Section 4.1, eq. EqnShapeCorrVel), on the uploaded mesh: w_out [D][N]
 * (double) receives each generator's velocity, the cell's fluid velocity
 * p/m (0 where m <= 0) plus chi times a pull towards the cell's centre of
 * mass s_i. With d = |s_i - r_i|, R_i = (3V/4pi)^(1/3) in 3D ((V/pi)^(1/2)
 * in 2D) and x = d/(eta R_i), the pull is 0 for x < 0.9, c_i (s_i - r_i)/d
 * for x >= 1.1 (c_i the cell's sound speed, 0 in a vacuum cell) and that
 * times (d - 0.9 eta R_i)/(0.2 eta R_i) in between; with dt_lloyd > 0,
 * (s_i - r_i)/dt_lloyd replaces c_i (s_i - r_i)/d (the paper's timestep
 * form; chi = 1 then moves every pulled generator onto its centre of mass
 * in dt_lloyd). The paper's usual choice is eta = 0.25, chi = 1. MM_E_ARG
 * for eta <= 0, chi < 0, dt_lloyd < 0 or non-finite values; MM_E_STATE
 * without a mesh. */
mm_status mm_mesh_velocity(mm_ctx *ctx, const double *Q, double eta, double chi, double dt_lloyd,
                           double *w_out);

/* The rate of change of every cell's volume implied by the uploaded mesh's
 * generator velocities (Section 3.3, eq. eqnvolchange): rate [N] (double)
 * = the sum over the cell's faces of A_f w_f . n_f, the face normal taken
 * out of the cell. MM_E_STATE without a mesh. */
mm_status mm_volume_rate(mm_ctx *ctx, double *rate);

/* Replace the uploaded mesh's generator velocities by mesh_vel [D][N]
 * (device, kept by reference like the mesh's arrays; for example the output
 * of mm_mesh_velocity) and recompute the face velocities and the side
 * records that depend on them, without re-sorting the mesh. Synchronises.
 * MM_E_MESH if a velocity is not finite (the context then has no mesh);
 * MM_E_STATE without a mesh. */
mm_status mm_mesh_set_velocity(mm_ctx *ctx, const double *mesh_vel);

/* An external static gravitational field for the uploaded mesh (Section
 * 5.2, the standard coupling): accel [D][N] (device, kept by reference
 * until the next mm_mesh_upload, which clears it) holds g_i = -grad Phi at
 * every cell; NULL switches the field off. With a field, the face-flux pass
 * adds (dt/2) g_K to each side's predicted velocity (not to faces that fall
 * back to unextrapolated states), and the update adds
 * (dt/2)(m^n + m^(n+1)) g_i to the momentum and (dt/2)(p^n + p^(n+1)).g_i
 * to the energy, dt being that of the last face-flux pass (mm_apply_update
 * returns MM_E_STATE if none has run since the upload). The field is held
 * fixed over the step. MM_E_STATE without a mesh. */
mm_status mm_set_gravity(mm_ctx *ctx, const double *accel);

/* Reflective walls by mirrored generators (the boundary of the paper's
 * Rayleigh-Taylor test, Section 8; the mirroring of Section 3.6,
 * boundary conditions). The uploaded mesh is the caller's
 * tessellation of the generators together with their mirror images across
 * each wall plane normal to coordinate axis `axis` (0 <= axis < D), so that
 * the cells of the images close the domain at the walls. ghost [n_ghost]
 * and src [n_ghost] (int32 device arrays, kept by reference until the next
 * mm_mesh_upload, which clears them, or the next mm_set_walls) name each
 * mirror cell and the cell it images. n_ghost = 0 removes the walls.
 * Before each step, mm_hydro_step sets every mirror cell's state to its
 * source's with the momentum along `axis` negated (every other row of Q,
 * the entropy row included, copied), so that each wall face carries a
 * symmetric Riemann problem; the caller's split path calls mm_reflect
 * before mm_gradients. The mirror cells are then cells like the others:
 * they are updated by the step and overwritten by the next reflection, and
 * sums over the domain exclude them. A field set with mm_set_gravity must
 * hold the mirrored field (its component along `axis` negated) at the
 * mirror cells. Checks the lists on the device and synchronises: MM_E_ARG
 * if n_ghost is negative or not below N, a pointer is NULL, `axis` is out
 * of range, an index is outside [0, N), a mirror cell is its own source,
 * listed twice or the source of another (the walls are then removed);
 * MM_E_STATE without a mesh. Ends a timeline (mm_tb_begin). */
mm_status mm_set_walls(mm_ctx *ctx, int64_t n_ghost, const int32_t *ghost, const int32_t *src, int32_t axis);

/* The reflection of mm_set_walls on Q ([nrow][N] device, nrow = D+2, or
 * D+3 with the entropy row), enqueued on the context's stream; nothing
 * without walls. MM_E_STATE without a mesh. */
mm_status mm_reflect(mm_ctx *ctx, double *Q);

/* ------------------------------------------------------------------------
 * Learned starting guess for the Newton iteration on the star pressure
 * (a 3 -> 64 -> 64 -> 1 ReLU network; not part of the paper's method, which
 * leaves the guess to its cited exact solver). The parameter vector is
 * MM_MLP_PARAMS floats on the device:
 *   W1 [3][64] (input-major), b1 [64], W2 [64][64] (input-major), b2 [64],
 *   w3 [64], b3 [1].
 * Inputs x = (ln(rho_R/rho_L)/5, ln(P_R/P_L)/5, (u_R - u_L)/(c_L + c_R)/2),
 * output y = predicted ln(p* / p_std) with p_std the standard guess, so the
 * learned guess is p = p_std exp(y). The guess only changes where Newton
 * starts: every face still converges to tolerance, and a face whose
 * iteration does not converge from it restarts from the standard guess.
 * ------------------------------------------------------------------------ */
#define MM_MLP_PARAMS 4481

/* Pack a trained parameter vector (device floats) into the context's
 * workspace in bf16 matrix-core operand order. With params.guess ==
 * MM_GUESS_LEARNED, later flux calls use it for faces outside the regime
 * where the standard guess is its primitive-variable estimate. Needs a
 * workspace (mm_set_workspace; mm_workspace_bytes(ctx, 2, 1) suffices). */
mm_status mm_mlp_load(mm_ctx *ctx, const float *params);

/* Fused bf16 inference of the loaded network on features X [n][3] -> Y [n]
 * (the same device code the flux kernels run; for tests). */
mm_status mm_mlp_infer(mm_ctx *ctx, int64_t n, const float *X, float *Y);

/* fp32 reference forward of a parameter vector: X [n][3] -> Y [n]. */
mm_status mm_mlp_forward(const float *params, int64_t n, const float *X, float *Y, void *stream);

/* Training: gradient of the loss sum_s (y_s - T_s)^2 / n_total over the n
 * samples X [n][3], T [n], written to grad [MM_MLP_PARAMS + 1] (the last
 * element is the loss). scratch is device memory of
 * mm_mlp_grad_scratch_bytes(n) bytes. Deterministic (fixed summation order). */
int64_t mm_mlp_grad_scratch_bytes(int64_t n);
mm_status mm_mlp_grad(const float *params, int64_t n, int64_t n_total, const float *X, const float *T,
                      void *scratch, float *grad, void *stream);

/* One Adam step (bias-corrected with step >= 1) on params from grad, with
 * first and second moment buffers m1, m2 [MM_MLP_PARAMS]. */
mm_status mm_mlp_adam(float *params, const float *grad, float *m1, float *m2, float lr, float beta1,
                      float beta2, float eps, int32_t step, void *stream);

/* n independent 1D Riemann problems, states [6][n] double (rho_L, u_L, P_L,
 * rho_R, u_R, P_R), solved exactly with the context's mode (MM_FP64: double;
 * MM_MIXED: float, hard problems re-solved in double by a second pass, in
 * chunks of 2^22 problems) and guess, sampled at
 * x/t = 0: out [n][5] double = (rho_F, u_F, P_F, p*, p_std), p* the star
 * pressure and p_std the standard starting guess (both -1 where the problem
 * has no star state: vacuum); iters [n] (optional) the Newton
 * iterations of each problem. Counts into the diagnostics. Needs a
 * workspace, not a mesh. */
mm_status mm_riemann_batch(mm_ctx *ctx, int64_t n, const double *states, double *out, int32_t *iters);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * batch as mm_riemann_batch without a context or workspace. params gives
 * mode, guess, gamma, Newton tolerances, iteration limit and stream (the
 * stream must belong to the current device; dim, cfl and the entropy and
 * timestep fields are ignored). The call's scratch -- the hard-problem
 * list of the float form and the packed network of the learned guess -- is
 * a fixed array of MM_NOALLOC_SCRATCH_BYTES in device memory, one per GPU,
 * held from the library's first call on that GPU until the process ends;
 * problems go through it in chunks of MM_NOALLOC_CHUNK, so any
 * n <= MM_NOALLOC_MAX_BATCH fits. The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); mlp_params (device float
 * [MM_MLP_PARAMS], required with MM_GUESS_LEARNED, else ignored) is packed
 * into the scratch on every call. Results equal mm_riemann_batch's for the
 * same params bit for bit; no diagnostics are counted. Calls that overlap
 * on one GPU (other streams, other threads) share the one scratch and
 * race: the caller orders them. MM_E_ARG for n < 1, n > MM_NOALLOC_MAX_BATCH,
 * null pointers or invalid params; MM_E_DEVICE if the scratch cannot be
 * found on the current device. */
#define MM_NOALLOC_CHUNK ((int64_t)1 << 20)
#define MM_NOALLOC_MAX_BATCH ((int64_t)1 << 32)
#define MM_NOALLOC_SCRATCH_BYTES ((int64_t)4243456) /* 4.05 MiB */
mm_status mm_riemann_batch_noalloc(const mm_params *params, int64_t n, const double *states, double *out,
                                   int32_t *iters, const float *mlp_params);

/* The face-frame Riemann inputs of every face of the uploaded mesh for a
 * step dt > 0 from double reconstruction records (MM_FP64 contexts only):
 * out [6][F] float = (rho_L, u_L, P_L, rho_R, u_R, P_R) after extrapolation,
 * u along the L->R normal. Harvests training problems from the method's own
 * runs. */
mm_status mm_face_states(mm_ctx *ctx, double dt, const void *recon, float *out);

/* Diagnostics accumulated since the last reset; synchronises. */
mm_status mm_get_diag(mm_ctx *ctx, mm_diag *out);
mm_status mm_reset_diag(mm_ctx *ctx);

/* ------------------------------------------------------------------------
 * Individual power-of-two timesteps (Section 7.2), contexts created with
 * steps = MM_STEPS_INDIVIDUAL, on the uploaded tessellation.
 *
 * Time runs in ticks of dt_max / 2^levels. Each cell sits in a bin b
 * (0 <= b <= levels) and takes steps of 2^b ticks that start at multiples
 * of 2^b. mm_tb_step performs one synchronisation point at the current
 * tick ti:
 *  - the cells whose step ends at ti recompute their primitive variables
 *    and gradients from Q (the others keep the records of their last
 *    active step) and choose a new bin: the largest b with
 *    dt_max 2^(b - levels) <= dt_i, where
 *      dt_i = cfl min(tau_i, R_i / (c_i + |v_i - w_i|)),
 *      tau_i = min over the face neighbours j of
 *              r_ij / (c_i + c_j - (v_i - v_j).(r_i - r_j)/r_ij)
 *    (eq. EqnTiStepIndividual with the minimum over the Voronoi neighbours;
 *    pairs whose signal speed is not positive set no bound). A cell may
 *    move down any number of bins but up by one only, and only when the
 *    higher bin starts a step at ti;
 *  - every face whose smaller step (the smaller bin of its two cells)
 *    starts at ti is integrated over that step: each side is predicted
 *    from its cell's record to the middle of the face's step and both
 *    cells exchange the time-integrated flux (conservative);
 *  - the timeline advances to the next tick at which a step ends (the
 *    next multiple of the smallest occupied bin's step).
 * A global step on a context (mm_hydro_step, mm_gradients), a mesh upload
 * or new generator velocities end the timeline (the cell records are
 * shared); mm_tb_step then returns MM_E_STATE until the next mm_tb_begin.
 * The tessellation stays fixed along the timeline; with moving generators
 * the caller rebuilds and re-uploads the mesh and begins a new timeline.
 * Static gravity and walls are not combined with it (MM_E_STATE).
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t tick;          /* the last point performed (ticks) */
    int64_t next_tick;     /* the next point */
    int64_t active_cells;  /* cells whose step started at tick */
    int64_t active_faces;  /* faces integrated at tick */
    int32_t min_bin;       /* occupied bins after that point */
    int32_t max_bin;
    int32_t sparse;        /* 1: that point found its faces from the active cells'
                              side lists (at most 1/8 of the cells due); 0: it
                              scanned every face. Same results either way. */
    int32_t points;        /* points performed by the call */
    int32_t sparse_points; /* of which sparse */
    int32_t reserved;
    int64_t total_cells;   /* active cells summed over the call's points */
    int64_t total_faces;   /* active faces summed over the call's points */
    double next_time;      /* next_tick dt_max / 2^levels */
} mm_tb_info;

/* Start a timeline at tick 0 with every cell due (all cells take their
 * bins from the criterion at the first point). 0 <= levels <= 30,
 * dt_max > 0 and finite (MM_E_ARG otherwise); MM_E_STATE without a mesh
 * or on a context not created with MM_STEPS_INDIVIDUAL. */
mm_status mm_tb_begin(mm_ctx *ctx, double dt_max, int32_t levels);

/* Up to max_points (>= 1) synchronisation points on Q ([D+2][N] device,
 * updated in place), stopping before the first point whose tick is at or
 * beyond until_tick: the points are enqueued without the host in between
 * (the timeline's tick and path live on the device; a point past the stop
 * tick does nothing), and the call synchronises once at the end. info
 * (host, may be NULL) receives the last point's summary and the call's
 * totals. MM_E_RANGE when an active cell's criterion is below one tick:
 * that point and every later one leave Q untouched, and the timeline has
 * ended (bins and records of that point's active cells have changed; begin
 * a new one). MM_E_NONFINITE when a point left a non-finite conserved value
 * (the timeline advances). */
mm_status mm_tb_advance(mm_ctx *ctx, double *Q, int64_t until_tick, int32_t max_points, mm_tb_info *info);

/* One synchronisation point: mm_tb_advance with no stop tick and one point. */
mm_status mm_tb_step(mm_ctx *ctx, double *Q, mm_tb_info *info);

/* Device copies of the timeline's per-cell bins [N] and the ticks at which
 * their current steps started [N] (either pointer may be NULL). Stream-
 * ordered, no synchronisation. MM_E_STATE without a timeline. */
mm_status mm_tb_state(mm_ctx *ctx, int8_t *bins, int64_t *trec);

/* Human-readable name of a status code. */
const char *mm_status_str(mm_status s);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
