// mm.hip -- libmm: the C ABI declared in include/mm.h, on gfx950.
//
// One hydro step (Section 3's step list, items (ii), (iii), (v), (vi),
// (vii)) on a tessellation the caller provides. Device work per step:
//   k_prim_cfl     per cell        Q -> primitives in the cell records,
//                                  per-block Courant minimum
//   k_grad_limit   lane group/cell limited gradients from the side records;
//                                  its block 0 the global timestep (stays on
//                                  the device)
//   k_face_flux*   per face        extrapolation, Riemann solve, lab-frame flux
//   k_update       lane group/cell segmented sum of the face fluxes
// Individual timesteps (Section 7.2, mm_tb_*) run one synchronisation point
// per call with the kernels of k_tb.hpp around list-driven gradient and
// flux passes.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/mm.h"
#include "common.hpp"
#include "k_cell.hpp"
#include "k_flux.hpp"
#include "k_learn.hpp"
#include "k_mesh.hpp"
#include "k_tb.hpp"
#include "k_update.hpp"
#include "k_walls.hpp"
#include "layout.hpp"

using namespace mm;

namespace {

inline int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

// Sub-list capacities of an individual-timestep context. The active-face
// list takes what either path appends to one sub-list: the face scan of
// dense points (list_cap of its grid) or, on sparse points, the sides of
// the cells that reach one active sub-list, estimated as 1.25 times their
// mean count plus 1024 (mm_tb_begin checks the exact sums and keeps to the
// dense path where they do not fit). The touched list also takes those
// cells themselves.
constexpr unsigned kTbGrid = 8 * kLists;   // the fixed grids of a point's list walks and scans
inline int64_t tb_cells_per_residue(int64_t n) { return (grid_for(n) + kLists - 1) / kLists * kBlock; }
inline int64_t tb_face_cap(int64_t n, int64_t nf) {
    const int64_t sparse = (int64_t)(1.25 * (2.0 * (double)nf / (double)n) * (double)tb_cells_per_residue(n)) + 1024;
    // the face scan: kTbGrid / kLists blocks per sub-list, each appending at
    // most kBlock faces per round
    const int64_t rounds = (nf + (int64_t)kTbGrid * kBlock - 1) / ((int64_t)kTbGrid * kBlock);
    const int64_t dense = (int64_t)kTbGrid / kLists * kBlock * rounds;
    return sparse > dense ? sparse : dense;
}
inline int64_t tb_touch_cap(int64_t n, int64_t nf) { return tb_face_cap(n, nf) + tb_cells_per_residue(n); }
inline int64_t split_ints(int64_t cap) { return (int64_t)kLists * kListPad + kLists * cap; }

inline unsigned plain_grid_n(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

struct Layout {
    int64_t flags, diag, mlp, dtdev, bhard, dtpart, bsum, off, cursor, ent, nbr;
    int64_t loff, roff, rface;              // the update's left ranges and right faces
    int64_t ekmax;                          // energy switch: largest kinetic energy per cell (float when mixed)
    int64_t srec, frec, wf64, rec, flux;    // double path (frec, wf64 always; flux: timelines only)
    int64_t srec32, mrec, wrel, rec32, hard, w0, w0part, coff32;   // mixed path
    int64_t tb_bin, tb_trec, tb_sig, tb_touch, tb_cells, tb_faces, tb_touched, tb_info;   // individual timesteps
    int64_t total;
};

// em: the entropy mode (0 off, MM_ENTROPY_MACH, MM_ENTROPY_ENERGY).
Layout make_layout(int D, int mode, int em, bool tb, int64_t n, int64_t nf) {
    const int NV = D + 2;
    const int FM = NV + (em == MM_ENTROPY_MACH ? 2 : (em ? 1 : 0));   // Rec<D, em>::FM
    const int REC = (D == 3) ? Lay<3>::REC : Lay<2>::REC;
    const int FREC = (D == 3) ? Lay<3>::FREC : Lay<2>::FREC;
    const int WS = (D == 3) ? Lay<3>::WSTRIDE : Lay<2>::WSTRIDE;
    Layout L;
    int64_t o = 0;
    auto take = [&](int64_t bytes) { int64_t at = o; o += align256(bytes); return at; };
    // fixed-size regions first: their offsets do not depend on the mesh
    L.flags = take(64 * sizeof(int32_t));
    L.diag = take(kDiagSlots * sizeof(DiagDev));
    L.mlp = take(sizeof(MlpPacked));
    L.dtdev = take(4 * sizeof(double));
    L.bhard = mode == MM_FP64 ? -1 : take(list_ints((kBatchChunk + kBlock - 1) / kBlock) * sizeof(int32_t));
    L.dtpart = take((int64_t)grid_for(n) * sizeof(double));
    int64_t bs = 0, m = n + 1;
    while (m > 1) { m = (m + 1023) / 1024; bs += m + 1; }
    L.bsum = take((bs + 4) * sizeof(int32_t));
    L.off = take((n + 1) * sizeof(int32_t));
    L.cursor = take((n > nf ? n : nf) * sizeof(int32_t));   // cursors, then each face's right slot
    L.ent = take(2 * nf * sizeof(int32_t));
    L.nbr = take(2 * nf * sizeof(int32_t));
    L.frec = take(nf * FREC * sizeof(double));
    L.wf64 = take(nf * WS * sizeof(double));
    L.loff = take((n + 1) * sizeof(int32_t));
    L.roff = take((n + 1) * sizeof(int32_t));
    L.rface = take(nf * sizeof(int32_t));
    L.flux = take(nf * FM * sizeof(double));
    L.ekmax = em == MM_ENTROPY_ENERGY ? take(n * sizeof(double)) : -1;
    L.srec = L.srec32 = L.mrec = L.wrel = L.rec32 = L.rec = L.hard = L.w0 = L.w0part = L.coff32 = -1;
    if (mode == MM_FP64) {
        L.srec = take(2 * nf * Lay<3>::SREC64 * sizeof(double));
        L.rec = take(n * REC * sizeof(double));
    } else {
        L.srec32 = take(2 * nf * Lay<3>::SREC32 * sizeof(float));
        L.w0 = take(4 * sizeof(double));
        L.w0part = take((int64_t)plain_grid_n(n) * 2 * 3 * sizeof(double));
        L.mrec = take(nf * Lay<3>::MREC * sizeof(float));
        L.wrel = take(nf * D * sizeof(float));
        L.rec32 = take(n * REC * sizeof(float));
        L.coff32 = take(D * n * sizeof(float));
        // with individual timesteps the hard faces of one face sub-list
        L.hard = take((tb ? split_ints(tb_face_cap(n, nf)) : list_ints(grid_for(nf))) * sizeof(int32_t));
    }
    L.tb_bin = L.tb_trec = L.tb_sig = L.tb_touch = L.tb_cells = L.tb_faces = L.tb_touched = L.tb_info = -1;
    if (tb) {
        L.tb_bin = take(n);
        L.tb_trec = take(n * sizeof(int64_t));
        L.tb_sig = take(n * (D + 2) * sizeof(double));
        L.tb_touch = take(n * sizeof(int32_t));
        L.tb_cells = take(list_ints(grid_for(n)) * sizeof(int32_t));
        L.tb_faces = take(split_ints(tb_face_cap(n, nf)) * sizeof(int32_t));
        L.tb_touched = take(split_ints(tb_touch_cap(n, nf)) * sizeof(int32_t));
        L.tb_info = take(TB_INFO_INTS * sizeof(int32_t));
    }
    L.total = o;
    return L;
}

}  // namespace

struct mm_ctx {
    mm_params p;
    int D = 3;
    char *ws = nullptr;
    int64_t ws_bytes = 0;
    bool have_mesh = false;
    bool mlp_ready = false;
    bool diag_ready = false;
    int64_t n = 0, nf = 0;
    uint64_t faces_done = 0, waves_done = 0;
    mm_mesh mesh;
    const double *accel = nullptr;        // static gravitational field [D][N], or none
    double w0h[3] = {0.0, 0.0, 0.0};      // mixed mode: W0 of the mesh's velocities (host copy)
    bool have_ek = false;                 // the energy switch's neighbour energies are in the workspace
    const double *last_dt_dev = nullptr;  // timestep of the last face-flux pass (device) ...
    double last_dt = 0.0;                 // ... or its value
    bool have_dt = false;
    struct Walls {      // mirror cells of reflective walls (caller's device lists)
        int64_t n = 0;
        const int32_t *ghost = nullptr, *src = nullptr;
        int32_t axis = 0;
    } walls;
    struct Timeline {   // host copies; the state itself is in the info block
        bool on = false;
        double dt_max = 0.0;
        int32_t levels = 0;
        int64_t ti = 0;           // as of the last synchronisation
        bool sparse_ok = false;   // the sparse path's appends fit the sub-lists
    } tb;
    Layout lay;
    hipStream_t st() const { return (hipStream_t)p.stream; }
    template <typename T> T *at(int64_t off) const { return (T *)(ws + off); }
};

#define MM_CHECK(expr)                                  \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return MM_E_DEVICE;       \
    } while (0)

#define MM_LAUNCH_CHECK() MM_CHECK(hipGetLastError())

// Fixed grid of the hard-face pass (it strides over a device-side list).
constexpr unsigned kHardGrid = 8 * kLists;   // walks of the split hard lists

static unsigned plain_grid(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Grid for the lane-group kernels: kBlock / GS cells per block.
static unsigned group_grid(int D, int64_t n) {
    const int64_t per = kBlock / (D == 3 ? Group<3>::GS : Group<2>::GS);
    int64_t b = (n + per - 1) / per;
    b = (b + kXcd - 1) / kXcd * kXcd;
    return (unsigned)b;
}

// The entry points keep C linkage from their declarations in mm.h.

const char *mm_status_str(mm_status s) {
    switch (s) {
        case MM_OK: return "ok";
        case MM_E_ARG: return "invalid argument";
        case MM_E_MESH: return "invalid mesh";
        case MM_E_DEVICE: return "HIP runtime error";
        case MM_E_STATE: return "no workspace or no mesh";
        case MM_E_WORKSPACE: return "workspace too small";
        case MM_E_NONFINITE: return "non-finite conserved state";
        case MM_E_RANGE: return "timestep criterion below the smallest step";
        default: return "unknown status";
    }
}

mm_status mm_create(const mm_params *params, mm_ctx **out) {
    if (!params || !out) return MM_E_ARG;
    *out = nullptr;
    if (params->dim != 2 && params->dim != 3) return MM_E_ARG;
    if (params->mode != MM_FP64 && params->mode != MM_MIXED) return MM_E_ARG;
    if (params->guess != MM_GUESS_STANDARD && params->guess != MM_GUESS_LEARNED) return MM_E_ARG;
    if (!(params->gamma > 1.0) || !(params->cfl > 0.0)) return MM_E_ARG;
    if (params->entropy != MM_ENTROPY_OFF && params->entropy != MM_ENTROPY_MACH &&
        params->entropy != MM_ENTROPY_ENERGY)
        return MM_E_ARG;
    if (params->entropy == MM_ENTROPY_ENERGY &&
        (!(params->alpha_s >= 0.0) || !(params->beta_s >= 0.0) || !isfinite(params->alpha_s) ||
         !isfinite(params->beta_s)))
        return MM_E_ARG;
    if (params->entropy != MM_ENTROPY_OFF && params->mach_thresh != params->mach_thresh) return MM_E_ARG;
    if (params->steps != MM_STEPS_GLOBAL && params->steps != MM_STEPS_INDIVIDUAL) return MM_E_ARG;
    if (params->steps == MM_STEPS_INDIVIDUAL && params->entropy != MM_ENTROPY_OFF) return MM_E_ARG;
    mm_ctx *c = new (std::nothrow) mm_ctx();
    if (!c) return MM_E_ARG;
    c->p = *params;
    if (c->p.newton_max_iter <= 0) c->p.newton_max_iter = 50;
    if (!(c->p.newton_tol64 > 0.0)) c->p.newton_tol64 = 1e-10;
    if (!(c->p.newton_tol32 > 0.0)) c->p.newton_tol32 = 1e-5;
    c->D = params->dim;
    *out = c;
    return MM_OK;
}

mm_status mm_destroy(mm_ctx *ctx) {
    delete ctx;
    return MM_OK;
}

int64_t mm_workspace_bytes(const mm_ctx *ctx, int64_t n_cells, int64_t n_faces) {
    if (!ctx || n_cells < 2 || n_faces < 1 || n_faces >= (int64_t(1) << 30) || n_cells >= (int64_t(1) << 31) - 1)
        return -1;
    return make_layout(ctx->D, ctx->p.mode, ctx->p.entropy, ctx->p.steps != 0, n_cells, n_faces).total;
}

mm_status mm_set_workspace(mm_ctx *ctx, void *dev_ptr, int64_t bytes) {
    if (!ctx || !dev_ptr || bytes <= 0 || ((uintptr_t)dev_ptr & 255)) return MM_E_ARG;
    ctx->ws = (char *)dev_ptr;
    ctx->ws_bytes = bytes;
    ctx->have_mesh = false;
    ctx->mlp_ready = false;
    ctx->diag_ready = false;
    // fixed-size regions (flags, diagnostics, network) sit at offsets that
    // no mesh changes
    ctx->lay = make_layout(ctx->D, ctx->p.mode, ctx->p.entropy, ctx->p.steps != 0, 2, 1);
    return MM_OK;
}

static mm_status clear_diag(mm_ctx *c) {
    // fill kernels rather than memset nodes, so callers may capture this
    const int64_t nd = kDiagSlots * sizeof(DiagDev) / sizeof(int32_t);
    k_fill_i32<<<plain_grid(nd), kBlock, 0, c->st()>>>(c->at<int32_t>(c->lay.diag), nd, 0);
    k_fill_i32<<<1, kBlock, 0, c->st()>>>(c->at<int32_t>(c->lay.flags) + 1, 2, 0);
    MM_LAUNCH_CHECK();
    c->faces_done = 0;
    c->waves_done = 0;
    c->diag_ready = true;
    return MM_OK;
}

// Workspace present and its fixed regions initialised.
static mm_status need_ws(mm_ctx *c) {
    if (!c->ws || c->ws_bytes < make_layout(c->D, c->p.mode, c->p.entropy, c->p.steps != 0, 2, 1).total) return MM_E_STATE;
    if (!c->diag_ready) return clear_diag(c);
    return MM_OK;
}

static const MlpPacked *active_mlp(const mm_ctx *c) {
    return (c->p.guess == MM_GUESS_LEARNED && c->mlp_ready) ? c->at<MlpPacked>(c->lay.mlp) : nullptr;
}

static mm_status scan_inclusive(mm_ctx *c, int32_t *data, int64_t n, int32_t *tile_sums) {
    const unsigned tiles = (unsigned)((n + 1023) / 1024);
    k_scan_tiles<<<tiles, kBlock, 0, c->st()>>>(data, n, tile_sums);
    MM_LAUNCH_CHECK();
    if (tiles > 1) {
        mm_status s = scan_inclusive(c, tile_sums, tiles, tile_sums + tiles + 1);
        if (s != MM_OK) return s;
        k_scan_add<<<tiles, kBlock, 0, c->st()>>>(data, n, tile_sums);
        MM_LAUNCH_CHECK();
    }
    return MM_OK;
}

template <int D> static void launch_validate(mm_ctx *c, const mm_mesh *m, int32_t *flags) {
    k_validate_faces<D><<<plain_grid(m->n_faces), kBlock, 0, c->st()>>>(
        m->n_cells, m->n_faces, m->face_L, m->face_R, m->face_area, m->face_ctr, m->face_sep, flags);
    k_validate_cells<D><<<plain_grid(m->n_cells), kBlock, 0, c->st()>>>(m->n_cells, m->volume, m->centroid_off,
                                                                        m->mesh_vel, flags);
}

// The mixed mode's reference velocity W0 (the midrange of the generator
// velocities) and the face records: everything that depends on the
// generator velocities; with so.ent (the upload) also the side records.
// The mixed mode's W0 into the context's host copy (the face kernels take it
// by value); complete at the caller's next synchronisation.
static mm_status fetch_w0(mm_ctx *c) {
    if (c->p.mode != MM_MIXED) return MM_OK;
    MM_CHECK(hipMemcpyAsync(c->w0h, c->at<double>(c->lay.w0), c->D * sizeof(double), hipMemcpyDeviceToHost, c->st()));
    return MM_OK;
}

template <int D> static void launch_face_records(mm_ctx *c, const mm_mesh *m, const SideOut &so = SideOut{}) {
    const Layout &L = c->lay;
    const int mixed = c->p.mode == MM_MIXED;
    if (mixed) {
        const unsigned g = plain_grid(m->n_cells);
        k_w0_part<D><<<g, kBlock, 0, c->st()>>>(m->n_cells, m->mesh_vel, c->at<double>(L.w0part));
        k_w0_final<D><<<1, kBlock, 0, c->st()>>>(g, c->at<double>(L.w0part), c->at<double>(L.w0));
    }
    k_face_records<D><<<plain_grid(m->n_faces), kBlock, 0, c->st()>>>(
        m->n_cells, m->n_faces, m->face_L, m->face_R, m->face_area, m->face_ctr, m->face_sep, m->mesh_vel,
        c->at<double>(L.frec), mixed ? c->at<double>(L.w0) : nullptr, mixed ? c->at<float>(L.mrec) : nullptr,
        mixed ? c->at<float>(L.wrel) : nullptr, c->at<double>(L.wf64), so);
}

mm_status mm_mesh_upload(mm_ctx *c, const mm_mesh *m) {
    if (!c || !m) return MM_E_ARG;
    if (!c->ws) return MM_E_STATE;
    const int64_t n = m->n_cells, nf = m->n_faces;
    if (n < 2 || nf < 1 || nf >= (int64_t(1) << 30) || n >= (int64_t(1) << 31) - 1) return MM_E_ARG;
    if (!m->volume || !m->centroid_off || !m->mesh_vel || !m->face_L || !m->face_R || !m->face_area ||
        !m->face_ctr || !m->face_sep)
        return MM_E_ARG;
    Layout L = make_layout(c->D, c->p.mode, c->p.entropy, c->p.steps != 0, n, nf);
    if (L.total > c->ws_bytes) return MM_E_WORKSPACE;
    c->have_mesh = false;
    c->tb.on = false;
    c->accel = nullptr;   // a field and walls belong to the mesh they were set for
    c->have_ek = false;
    c->walls = mm_ctx::Walls();
    c->have_dt = false;
    c->lay = L;
    c->n = n;
    c->nf = nf;
    c->mesh = *m;
    hipStream_t s = c->st();
    int32_t *flags = c->at<int32_t>(L.flags);
    k_fill_i32<<<1, kBlock, 0, s>>>(flags, 64, 0);
    MM_LAUNCH_CHECK();
    if (c->D == 3) launch_validate<3>(c, m, flags);
    else launch_validate<2>(c, m, flags);
    MM_LAUNCH_CHECK();
    int32_t hflags = 0;
    MM_CHECK(hipMemcpyAsync(&hflags, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MM_CHECK(hipStreamSynchronize(s));
    if (hflags) return MM_E_MESH;

    // each cell's left range (faces are sorted by left cell) and its right
    // faces in ascending face order
    int32_t *off = c->at<int32_t>(L.off), *cur = c->at<int32_t>(L.cursor);
    int32_t *loff = c->at<int32_t>(L.loff), *roff = c->at<int32_t>(L.roff), *rface = c->at<int32_t>(L.rface);
    k_left_offsets<<<plain_grid(n + 1), kBlock, 0, s>>>(n, nf, m->face_L, loff);
    k_fill_i32<<<plain_grid(n + 1), kBlock, 0, s>>>(roff, n + 1, 0);
    k_count_right<<<plain_grid(nf), kBlock, 0, s>>>(nf, m->face_R, roff + 1);
    MM_LAUNCH_CHECK();
    mm_status st = scan_inclusive(c, roff + 1, n, c->at<int32_t>(L.bsum));
    if (st != MM_OK) return st;
    k_copy_i32<<<plain_grid(n), kBlock, 0, s>>>(cur, roff, n);
    k_place_right<<<plain_grid(nf), kBlock, 0, s>>>(nf, m->face_R, cur, rface);
    int32_t *pos = cur;   // the cursors are spent: each face's slot in rface
    k_sort_right<<<plain_grid(n), kBlock, 0, s>>>(n, roff, rface, pos);
    MM_LAUNCH_CHECK();
    // the face records and face velocities; from them the gradient pass's
    // side lists and records, and the closure test
    const bool mixed = c->p.mode == MM_MIXED;
    double *srec = mixed ? nullptr : c->at<double>(L.srec);
    float *srec32 = mixed ? c->at<float>(L.srec32) : nullptr;
    const SideOut so{loff, roff, pos, c->at<int32_t>(L.ent), c->at<int32_t>(L.nbr), srec, srec32};
    if (c->D == 3) {
        launch_face_records<3>(c, m, so);
        k_closure<3><<<group_grid(3, n), kBlock, 0, s>>>(n, c->at<double>(L.frec), loff, roff, rface, off, flags);
        if (mixed) k_coff32<3><<<plain_grid(n), kBlock, 0, s>>>(n, m->centroid_off, c->at<float>(L.coff32));
    } else {
        launch_face_records<2>(c, m, so);
        k_closure<2><<<group_grid(2, n), kBlock, 0, s>>>(n, c->at<double>(L.frec), loff, roff, rface, off, flags);
        if (mixed) k_coff32<2><<<plain_grid(n), kBlock, 0, s>>>(n, m->centroid_off, c->at<float>(L.coff32));
    }
    MM_LAUNCH_CHECK();
    if (mm_status st = fetch_w0(c); st != MM_OK) return st;
    MM_CHECK(hipMemcpyAsync(&hflags, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MM_CHECK(hipStreamSynchronize(s));
    if (hflags) return MM_E_MESH;
    c->have_mesh = true;
    return clear_diag(c);
}

mm_status mm_mesh_set_velocity(mm_ctx *c, const double *mesh_vel) {
    if (!c || !mesh_vel) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    c->have_mesh = false;
    c->tb.on = false;
    c->mesh.mesh_vel = mesh_vel;
    const mm_mesh *m = &c->mesh;
    hipStream_t s = c->st();
    int32_t *flags = c->at<int32_t>(c->lay.flags);
    k_fill_i32<<<1, kBlock, 0, s>>>(flags, 1, 0);
    if (c->D == 3) {
        k_validate_cells<3><<<plain_grid(m->n_cells), kBlock, 0, s>>>(m->n_cells, m->volume, m->centroid_off,
                                                                      m->mesh_vel, flags);
        launch_face_records<3>(c, m);
    } else {
        k_validate_cells<2><<<plain_grid(m->n_cells), kBlock, 0, s>>>(m->n_cells, m->volume, m->centroid_off,
                                                                      m->mesh_vel, flags);
        launch_face_records<2>(c, m);
    }
    MM_LAUNCH_CHECK();
    int32_t hflags = 0;
    if (mm_status st = fetch_w0(c); st != MM_OK) return st;
    MM_CHECK(hipMemcpyAsync(&hflags, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MM_CHECK(hipStreamSynchronize(s));
    if (hflags) return MM_E_MESH;
    c->have_mesh = true;
    return MM_OK;
}

// The reconstruction buffer holds the primitive block [N][PREC] followed by
// the gradient block [N][GREC].
template <int D, typename T> static T *grad_block(const mm_ctx *c, T *rec) { return rec + c->n * Lay<D>::PREC; }

// What the step's own gradient pass does besides: clear the face pass's
// hard-list counters (clear), and reduce the Courant minima to the
// timestep on the device (dt_out).
struct StepPass {
    int32_t *clear = nullptr;
    double *dt_out = nullptr;
};

template <int D, typename T>
static mm_status gradients_t(mm_ctx *c, const double *Q, T *rec, double *dt_part, const StepPass &sp) {
    const Layout &L = c->lay;
    hipStream_t s = c->st();
    const bool f64 = sizeof(T) == 8;
    const T *srec = f64 ? (const T *)c->at<double>(L.srec) : (const T *)c->at<float>(L.srec32);
    const double *w0 = f64 ? nullptr : c->at<double>(L.w0);
    const T *coff = f64 ? (const T *)c->mesh.centroid_off : (const T *)c->at<float>(L.coff32);
    const unsigned pg = grid_for(c->n);
    k_prim_cfl<D, T><<<pg, kBlock, 0, s>>>(c->n, c->p.gamma, c->p.cfl, c->mesh.volume, Q, c->mesh.mesh_vel, coff,
                                          rec, w0, dt_part, c->at<int32_t>(L.flags) + 2, sp.clear,
                                          sp.clear ? kLists * kListPad : 0);
    if (c->p.entropy == MM_ENTROPY_ENERGY) {   // with the energy switch's neighbour energies
        k_grad_limit<D, T, true><<<group_grid(D, c->n), kBlock, 0, s>>>(
            c->n, c->at<int32_t>(L.off), c->at<int32_t>(L.nbr), srec, c->mesh.volume, rec, grad_block<D>(c, rec),
            c->mesh.mesh_vel, w0, (T *)c->at<double>(L.ekmax), dt_part, pg, sp.dt_out);
        c->have_ek = true;
    } else {
        k_grad_limit<D, T, false><<<group_grid(D, c->n), kBlock, 0, s>>>(
            c->n, c->at<int32_t>(L.off), c->at<int32_t>(L.nbr), srec, c->mesh.volume, rec, grad_block<D>(c, rec),
            nullptr, nullptr, nullptr, dt_part, pg, sp.dt_out);
    }
    MM_LAUNCH_CHECK();
    return MM_OK;
}

static mm_status gradients_into(mm_ctx *c, const double *Q, void *rec, double *dt_part, const StepPass &sp = {}) {
    const bool f64 = c->p.mode == MM_FP64;
    if (c->D == 3)
        return f64 ? gradients_t<3, double>(c, Q, (double *)rec, dt_part, sp)
                   : gradients_t<3, float>(c, Q, (float *)rec, dt_part, sp);
    return f64 ? gradients_t<2, double>(c, Q, (double *)rec, dt_part, sp)
               : gradients_t<2, float>(c, Q, (float *)rec, dt_part, sp);
}

mm_status mm_gradients(mm_ctx *c, const double *Q, void *recon) {
    if (!c || !Q || !recon) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    c->tb.on = false;
    return gradients_into(c, Q, recon, c->at<double>(c->lay.dtpart));
}

static FaceAux face_aux(const mm_ctx *c) {
    const bool mixed = c->p.mode == MM_MIXED;
    return FaceAux{c->accel, c->n, {c->w0h[0], c->w0h[1], c->w0h[2]}, mixed ? c->at<float>(c->lay.wrel) : nullptr};
}

// The face fluxes in entropy mode EM, face-major records into flux.
template <int D, int EM, bool GRAV>
static mm_status fluxes_t(mm_ctx *c, const double *dt_dev, double dt, const void *rec, double *flux, bool cleared) {
    const Layout &L = c->lay;
    hipStream_t s = c->st();
    DiagDev *diag = c->at<DiagDev>(L.diag);
    const MlpPacked *mlp = active_mlp(c);
    const GasConst<double> kg(c->p.gamma);
    const GasConst<float> kf(c->p.gamma);
    const FaceAux aux = face_aux(c);
    if (c->p.mode == MM_FP64) {
        auto kern = mlp ? k_face_flux64<D, true, EM, GRAV> : k_face_flux64<D, false, EM, GRAV>;
        const double *prim = (const double *)rec;
        kern<<<grid_for(c->nf), kBlock, 0, s>>>(c->nf, c->mesh.face_L, c->mesh.face_R, c->at<double>(L.frec),
                                                c->at<double>(L.wf64), prim,
                                                grad_block<D>(c, prim), dt_dev, dt, kg, c->p.newton_tol64,
                                                c->p.newton_max_iter, mlp, flux, diag, aux);
    } else {
        int32_t *hard = c->at<int32_t>(L.hard);
        const int64_t cap = list_cap(grid_for(c->nf));
        if (!cleared)   // (the step's gradient pass has done it)
            k_fill_i32<<<kLists * kListPad / kBlock, kBlock, 0, s>>>(hard, kLists * kListPad, 0);
        auto kern = mlp ? k_face_flux_mixed<D, true, EM, GRAV> : k_face_flux_mixed<D, false, EM, GRAV>;
        const float *prim = (const float *)rec;
        kern<<<grid_for(c->nf), kBlock, 0, s>>>(c->nf, c->mesh.face_L, c->mesh.face_R, c->at<float>(L.mrec), prim,
                                                grad_block<D>(c, prim), dt_dev, dt, kf,
                                                kg.g_over_gm1, (float)c->p.newton_tol32, c->p.newton_max_iter, mlp,
                                                flux, hard, cap, diag, aux);
        k_face_flux_hard<D, EM, GRAV><<<kHardGrid, kBlock, 0, s>>>(
            c->mesh.face_L, c->mesh.face_R, c->at<float>(L.mrec), prim, grad_block<D>(c, prim),
            dt_dev, dt, kf.g, kg, c->p.newton_tol64, hard, cap, flux, diag, aux, TbView{});
    }
    MM_LAUNCH_CHECK();
    return MM_OK;
}

template <int D>
static mm_status fluxes_d(mm_ctx *c, const double *dt_dev, double dt, const void *rec, double *flux, bool cleared) {
    const bool g = c->accel != nullptr;
    switch (c->p.entropy) {
        case MM_ENTROPY_MACH:
            return g ? fluxes_t<D, 1, true>(c, dt_dev, dt, rec, flux, cleared)
                     : fluxes_t<D, 1, false>(c, dt_dev, dt, rec, flux, cleared);
        case MM_ENTROPY_ENERGY:   // the entropy flux without the Mach number
            return g ? fluxes_t<D, 2, true>(c, dt_dev, dt, rec, flux, cleared)
                     : fluxes_t<D, 2, false>(c, dt_dev, dt, rec, flux, cleared);
        default:
            return g ? fluxes_t<D, 0, true>(c, dt_dev, dt, rec, flux, cleared)
                     : fluxes_t<D, 0, false>(c, dt_dev, dt, rec, flux, cleared);
    }
}

static mm_status fluxes_into(mm_ctx *c, const double *dt_dev, double dt, const void *rec, double *flux,
                             bool cleared = false) {
    c->faces_done += (uint64_t)c->nf;
    c->waves_done += (uint64_t)((c->nf + 63) / 64);
    c->last_dt_dev = dt_dev;
    c->last_dt = dt;
    c->have_dt = true;
    return c->D == 3 ? fluxes_d<3>(c, dt_dev, dt, rec, flux, cleared) : fluxes_d<2>(c, dt_dev, dt, rec, flux, cleared);
}

mm_status mm_face_fluxes(mm_ctx *c, double dt, const void *recon, double *face_flux) {
    if (!c || !recon || !face_flux) return MM_E_ARG;
    if (!(dt > 0.0) || !isfinite(dt)) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    return fluxes_into(c, nullptr, dt, recon, face_flux);
}

static UpdateArgs update_args(const mm_ctx *c) {
    const Layout &L = c->lay;
    return UpdateArgs{c->at<int32_t>(L.flags) + 1, c->mesh.volume, c->p.gamma, c->p.mach_thresh,
                      c->at<DiagDev>(L.diag), c->accel, c->last_dt_dev, c->last_dt, c->p.alpha_s, c->p.beta_s,
                      (L.ekmax >= 0 && c->p.mode == MM_FP64) ? c->at<double>(L.ekmax) : nullptr,
                      (L.ekmax >= 0 && c->p.mode == MM_MIXED) ? c->at<float>(L.ekmax) : nullptr};
}

// The update from face-major records.
template <int D, int EM, bool GRAV> static void launch_update(mm_ctx *c, const double *flux, double *Q) {
    const Layout &L = c->lay;
    k_update<D, EM, GRAV><<<group_grid(D, c->n), kBlock, 0, c->st()>>>(
        c->n, c->at<int32_t>(L.loff), c->at<int32_t>(L.roff), c->at<int32_t>(L.rface), flux, Q, update_args(c));
}

template <int D> static void launch_update_d(mm_ctx *c, const double *flux, double *Q) {
    const bool g = c->accel != nullptr;
    switch (c->p.entropy) {
        case MM_ENTROPY_MACH: g ? launch_update<D, 1, true>(c, flux, Q) : launch_update<D, 1, false>(c, flux, Q); break;
        case MM_ENTROPY_ENERGY: g ? launch_update<D, 2, true>(c, flux, Q) : launch_update<D, 2, false>(c, flux, Q); break;
        default: g ? launch_update<D, 0, true>(c, flux, Q) : launch_update<D, 0, false>(c, flux, Q);
    }
}

static mm_status update_into(mm_ctx *c, const double *flux, double *Q) {
    if (c->accel && !c->have_dt) return MM_E_STATE;   // the source terms need the flux pass's timestep
    if (c->p.entropy == MM_ENTROPY_ENERGY && !c->have_ek) return MM_E_STATE;   // no gradient pass yet
    if (c->D == 3) launch_update_d<3>(c, flux, Q);
    else launch_update_d<2>(c, flux, Q);
    MM_LAUNCH_CHECK();
    return MM_OK;
}

mm_status mm_set_gravity(mm_ctx *c, const double *accel) {
    if (!c) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    c->accel = accel;
    return MM_OK;
}

static int row_count(const mm_ctx *c) { return c->D + 2 + (c->p.entropy ? 1 : 0); }

static void launch_reflect(mm_ctx *c, double *Q) {
    k_reflect<<<plain_grid(c->walls.n), kBlock, 0, c->st()>>>(c->n, c->walls.n, row_count(c), c->walls.axis,
                                                              c->walls.ghost, c->walls.src, Q);
}

mm_status mm_set_walls(mm_ctx *c, int64_t n_ghost, const int32_t *ghost, const int32_t *src, int32_t axis) {
    if (!c) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    if (n_ghost < 0 || n_ghost >= c->n) return MM_E_ARG;
    c->walls = mm_ctx::Walls();
    c->tb.on = false;   // a timeline does not reflect
    if (n_ghost == 0) return MM_OK;
    if (!ghost || !src || axis < 0 || axis >= c->D) return MM_E_ARG;
    const Layout &L = c->lay;
    hipStream_t s = c->st();
    int32_t *flag = c->at<int32_t>(L.flags) + 8;
    int32_t *mark = c->at<int32_t>(L.cursor);   // free after the upload
    k_fill_i32<<<1, kBlock, 0, s>>>(flag, 1, 0);
    k_fill_i32<<<plain_grid(c->n), kBlock, 0, s>>>(mark, c->n, 0);
    k_walls_mark<<<plain_grid(n_ghost), kBlock, 0, s>>>(c->n, n_ghost, ghost, src, mark, flag);
    k_walls_check<<<plain_grid(n_ghost), kBlock, 0, s>>>(c->n, n_ghost, ghost, src, mark, flag);
    MM_LAUNCH_CHECK();
    int32_t bad = 0;
    MM_CHECK(hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MM_CHECK(hipStreamSynchronize(s));
    if (bad) return MM_E_ARG;
    c->walls.n = n_ghost;
    c->walls.ghost = ghost;
    c->walls.src = src;
    c->walls.axis = axis;
    return MM_OK;
}

mm_status mm_reflect(mm_ctx *c, double *Q) {
    if (!c || !Q) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    if (!c->walls.n) return MM_OK;
    launch_reflect(c, Q);
    MM_LAUNCH_CHECK();
    return MM_OK;
}

mm_status mm_mesh_velocity(mm_ctx *c, const double *Q, double eta, double chi, double dt_lloyd, double *w_out) {
    if (!c || !Q || !w_out) return MM_E_ARG;
    if (!(eta > 0.0) || !(chi >= 0.0) || !isfinite(eta) || !isfinite(chi) || !(dt_lloyd >= 0.0) || !isfinite(dt_lloyd))
        return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    if (c->D == 3)
        k_mesh_velocity<3><<<plain_grid(c->n), kBlock, 0, c->st()>>>(c->n, Q, c->mesh.volume, c->mesh.centroid_off,
                                                                     c->p.gamma, eta, chi, dt_lloyd, w_out);
    else
        k_mesh_velocity<2><<<plain_grid(c->n), kBlock, 0, c->st()>>>(c->n, Q, c->mesh.volume, c->mesh.centroid_off,
                                                                     c->p.gamma, eta, chi, dt_lloyd, w_out);
    MM_LAUNCH_CHECK();
    return MM_OK;
}

mm_status mm_volume_rate(mm_ctx *c, double *rate) {
    if (!c || !rate) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    const Layout &L = c->lay;
    if (c->D == 3)
        k_volume_rate<3><<<group_grid(3, c->n), kBlock, 0, c->st()>>>(c->n, c->at<int32_t>(L.off),
                                                                      c->at<int32_t>(L.ent), c->at<double>(L.frec),
                                                                      c->at<double>(L.wf64), rate);
    else
        k_volume_rate<2><<<group_grid(2, c->n), kBlock, 0, c->st()>>>(c->n, c->at<int32_t>(L.off),
                                                                      c->at<int32_t>(L.ent), c->at<double>(L.frec),
                                                                      c->at<double>(L.wf64), rate);
    MM_LAUNCH_CHECK();
    return MM_OK;
}

mm_status mm_entropy_init(mm_ctx *c, double *Q) {
    if (!c || !Q) return MM_E_ARG;
    if (!c->p.entropy) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    if (c->D == 3) k_entropy_init<3><<<plain_grid(c->n), kBlock, 0, c->st()>>>(c->n, c->mesh.volume, c->p.gamma, Q);
    else k_entropy_init<2><<<plain_grid(c->n), kBlock, 0, c->st()>>>(c->n, c->mesh.volume, c->p.gamma, Q);
    MM_LAUNCH_CHECK();
    return MM_OK;
}

mm_status mm_apply_update(mm_ctx *c, const double *face_flux, double *Q) {
    if (!c || !face_flux || !Q) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    return update_into(c, face_flux, Q);
}

mm_status mm_hydro_step(mm_ctx *c, double *Q, double dt, double *dt_used) {
    if (!c || !Q) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    if (!isfinite(dt)) return MM_E_ARG;
    c->tb.on = false;   // the step rewrites the cell records a timeline keeps
    const Layout &L = c->lay;
    hipStream_t s = c->st();
    if (c->walls.n) {
        launch_reflect(c, Q);
        MM_LAUNCH_CHECK();
    }
    void *rec = c->p.mode == MM_FP64 ? (void *)c->at<double>(L.rec) : (void *)c->at<float>(L.rec32);
    double *dt_part = c->at<double>(L.dtpart);
    double *dt_dev = c->at<double>(L.dtdev);
    StepPass sp;
    if (c->p.mode == MM_MIXED) sp.clear = c->at<int32_t>(L.hard);
    if (!(dt > 0.0)) sp.dt_out = dt_dev;   // the Courant step
    mm_status st = gradients_into(c, Q, rec, dt_part, sp);
    if (st != MM_OK) return st;
    const double *dt_src = sp.dt_out;
    double *flux = c->at<double>(L.flux);
    st = fluxes_into(c, dt_src, dt, rec, flux, sp.clear != nullptr);
    if (st != MM_OK) return st;
    st = update_into(c, flux, Q);
    if (st != MM_OK) return st;
    if (dt_used) {
        int32_t nonfin = 0;
        if (dt_src) MM_CHECK(hipMemcpyAsync(dt_used, dt_dev, sizeof(double), hipMemcpyDeviceToHost, s));
        else *dt_used = dt;
        MM_CHECK(hipMemcpyAsync(&nonfin, c->at<int32_t>(L.flags) + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        MM_CHECK(hipStreamSynchronize(s));
        if (nonfin) return MM_E_NONFINITE;
    }
    return MM_OK;
}

mm_status mm_reset_diag(mm_ctx *c) {
    if (!c) return MM_E_ARG;
    if (!c->ws) return MM_E_STATE;
    return clear_diag(c);
}

mm_status mm_mlp_load(mm_ctx *c, const float *params) {
    if (!c || !params) return MM_E_ARG;
    mm_status st = need_ws(c);
    if (st != MM_OK) return st;
    k_mlp_pack<<<1, kBlock, 0, c->st()>>>(params, c->at<MlpPacked>(c->lay.mlp));
    MM_LAUNCH_CHECK();
    c->mlp_ready = true;
    return MM_OK;
}

mm_status mm_mlp_infer(mm_ctx *c, int64_t n, const float *X, float *Y) {
    if (!c || !X || !Y || n < 1) return MM_E_ARG;
    if (!c->mlp_ready) return MM_E_STATE;
    k_mlp_infer<<<plain_grid(n), kBlock, 0, c->st()>>>(n, c->at<MlpPacked>(c->lay.mlp), X, Y);
    MM_LAUNCH_CHECK();
    return MM_OK;
}

mm_status mm_mlp_forward(const float *params, int64_t n, const float *X, float *Y, void *stream) {
    if (!params || !X || !Y || n < 1) return MM_E_ARG;
    k_mlp_forward<<<plain_grid(n), kBlock, 0, (hipStream_t)stream>>>(n, params, X, Y);
    MM_LAUNCH_CHECK();
    return MM_OK;
}

int64_t mm_mlp_grad_scratch_bytes(int64_t n) {
    if (n < 1) return -1;
    return ((n + kMlpTile - 1) / kMlpTile) * (int64_t)(kMlpParams + 1) * (int64_t)sizeof(float);
}

mm_status mm_mlp_grad(const float *params, int64_t n, int64_t n_total, const float *X, const float *T, void *partials,
                      float *grad, void *stream) {
    if (!params || !X || !T || !partials || !grad || n < 1 || n_total < 1) return MM_E_ARG;
    const int64_t nb = (n + kMlpTile - 1) / kMlpTile;
    hipStream_t s = (hipStream_t)stream;
    k_mlp_grad_partial<<<(unsigned)nb, kBlock, 0, s>>>(n, 1.0f / (float)n_total, params, X, T, (float *)partials);
    k_mlp_reduce<<<plain_grid(kMlpParams + 1), kBlock, 0, s>>>(nb, (const float *)partials, grad);
    MM_LAUNCH_CHECK();
    return MM_OK;
}

mm_status mm_mlp_adam(float *params, const float *grad, float *m1, float *m2, float lr, float beta1, float beta2,
                      float eps, int32_t step, void *stream) {
    if (!params || !grad || !m1 || !m2 || step < 1) return MM_E_ARG;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    k_mlp_adam<<<plain_grid(kMlpParams), kBlock, 0, (hipStream_t)stream>>>(params, grad, m1, m2, lr, beta1, beta2, eps,
                                                                          c1, c2);
    MM_LAUNCH_CHECK();
    return MM_OK;
}

mm_status mm_riemann_batch(mm_ctx *c, int64_t n, const double *states, double *out, int32_t *iters) {
    if (!c || !states || !out || n < 1) return MM_E_ARG;
    mm_status st = need_ws(c);
    if (st != MM_OK) return st;
    DiagDev *diag = c->at<DiagDev>(c->lay.diag);
    const MlpPacked *mlp = active_mlp(c);
    const GasConst<double> kg(c->p.gamma);
    c->faces_done += (uint64_t)n;
    c->waves_done += (uint64_t)((n + 63) / 64);
    for (int64_t i0 = 0; i0 < n; i0 += kBatchChunk) {
        const int64_t nc = n - i0 < kBatchChunk ? n - i0 : kBatchChunk;
        if (c->p.mode == MM_FP64) {
            auto kern = mlp ? k_riemann_batch<double, true> : k_riemann_batch<double, false>;
            kern<<<plain_grid(nc), kBlock, 0, c->st()>>>(n, i0, nc, states, kg, c->p.newton_tol64,
                                                         c->p.newton_max_iter, mlp, out, iters, nullptr, 0, diag);
        } else {
            int32_t *hard = c->at<int32_t>(c->lay.bhard);
            const int64_t cap = list_cap(plain_grid(nc));
            k_fill_i32<<<kLists * kListPad / kBlock, kBlock, 0, c->st()>>>(hard, kLists * kListPad, 0);
            auto kern = mlp ? k_riemann_batch<float, true> : k_riemann_batch<float, false>;
            kern<<<plain_grid(nc), kBlock, 0, c->st()>>>(n, i0, nc, states, GasConst<float>(c->p.gamma),
                                                         (float)c->p.newton_tol32, c->p.newton_max_iter, mlp, out,
                                                         iters, hard, cap, diag);
            k_riemann_hard<<<kHardGrid, kBlock, 0, c->st()>>>(n, i0, states, kg, c->p.newton_tol64, hard, cap, out,
                                                              iters, diag);
        }
    }
    MM_LAUNCH_CHECK();
    return MM_OK;
}

// ------------------------------------------------------------------------
// The batch without a context (mm_riemann_batch_noalloc): its scratch is a
// fixed array in device memory, one copy per GPU. Host code never passes the
// array's name to a kernel or a copy (in host code it names a host-side
// stand-in); it uses the device address that hipGetSymbolAddress returns for
// the current device, looked up once per device and kept.
namespace {

constexpr int64_t kNoAllocHardInts = (int64_t)kLists * kListPad + (int64_t)kLists * ((MM_NOALLOC_CHUNK / kBlock + kLists - 1) / kLists * kBlock);
constexpr int64_t kNoAllocMlpOff = (kNoAllocHardInts * 4 + 255) / 256 * 256;   // bytes
static_assert(kNoAllocMlpOff + (int64_t)sizeof(MlpPacked) <= MM_NOALLOC_SCRATCH_BYTES, "scratch too small");
static_assert(MM_NOALLOC_SCRATCH_BYTES % 4 == 0, "scratch of whole words");

__device__ __align__(256) int32_t scratch[MM_NOALLOC_SCRATCH_BYTES / 4];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The scratch's device address on the current device (nullptr on failure).
void *scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

mm_status mm_riemann_batch_noalloc(const mm_params *params, int64_t n, const double *states, double *out,
                                   int32_t *iters, const float *mlp_params) {
    if (!params || !states || !out || n < 1 || n > MM_NOALLOC_MAX_BATCH) return MM_E_ARG;
    if (params->mode != MM_FP64 && params->mode != MM_MIXED) return MM_E_ARG;
    if (params->guess != MM_GUESS_STANDARD && params->guess != MM_GUESS_LEARNED) return MM_E_ARG;
    if (params->guess == MM_GUESS_LEARNED && !mlp_params) return MM_E_ARG;
    if (!(params->gamma > 1.0) || !isfinite(params->gamma)) return MM_E_ARG;
    // the context's defaults for unset solver parameters (mm_create)
    const int maxit = params->newton_max_iter > 0 ? params->newton_max_iter : 50;
    const double tol64 = params->newton_tol64 > 0.0 ? params->newton_tol64 : 1e-10;
    const double tol32 = params->newton_tol32 > 0.0 ? params->newton_tol32 : 1e-5;
    char *sp = (char *)scratch_on_current_device();
    if (!sp) return MM_E_DEVICE;
    hipStream_t s = (hipStream_t)params->stream;
    int32_t *hard = (int32_t *)sp;
    MlpPacked *mlp = nullptr;
    if (params->guess == MM_GUESS_LEARNED) {
        mlp = (MlpPacked *)(sp + kNoAllocMlpOff);
        k_mlp_pack<<<1, kBlock, 0, s>>>(mlp_params, mlp);
    }
    const GasConst<double> kg(params->gamma);
    for (int64_t i0 = 0; i0 < n; i0 += MM_NOALLOC_CHUNK) {
        const int64_t nc = n - i0 < MM_NOALLOC_CHUNK ? n - i0 : MM_NOALLOC_CHUNK;
        if (params->mode == MM_FP64) {
            auto kern = mlp ? k_riemann_batch<double, true> : k_riemann_batch<double, false>;
            kern<<<plain_grid(nc), kBlock, 0, s>>>(n, i0, nc, states, kg, tol64, maxit, mlp, out, iters, nullptr, 0,
                                                   nullptr);
        } else {
            const int64_t cap = list_cap(plain_grid(nc));
            // the list counters start at zero for every chunk (a fill kernel,
            // so that the call can be captured)
            k_fill_i32<<<kLists * kListPad / kBlock, kBlock, 0, s>>>(hard, kLists * kListPad, 0);
            auto kern = mlp ? k_riemann_batch<float, true> : k_riemann_batch<float, false>;
            kern<<<plain_grid(nc), kBlock, 0, s>>>(n, i0, nc, states, GasConst<float>(params->gamma), (float)tol32,
                                                   maxit, mlp, out, iters, hard, cap, nullptr);
            k_riemann_hard<<<kHardGrid, kBlock, 0, s>>>(n, i0, states, kg, tol64, hard, cap, out, iters, nullptr);
        }
    }
    MM_LAUNCH_CHECK();
    return MM_OK;
}

mm_status mm_face_states(mm_ctx *c, double dt, const void *recon, float *out) {
    if (!c || !recon || !out || !(dt > 0.0) || !isfinite(dt)) return MM_E_ARG;
    if (c->p.mode != MM_FP64) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    if (c->D == 3)
        k_face_states64<3><<<plain_grid(c->nf), kBlock, 0, c->st()>>>(
            c->nf, c->mesh.face_L, c->mesh.face_R, c->at<double>(c->lay.frec), c->at<double>(c->lay.wf64),
            (const double *)recon,
            grad_block<3>(c, (const double *)recon), dt, c->p.gamma, out);
    else
        k_face_states64<2><<<plain_grid(c->nf), kBlock, 0, c->st()>>>(
            c->nf, c->mesh.face_L, c->mesh.face_R, c->at<double>(c->lay.frec), c->at<double>(c->lay.wf64),
            (const double *)recon,
            grad_block<2>(c, (const double *)recon), dt, c->p.gamma, out);
    MM_LAUNCH_CHECK();
    return MM_OK;
}

mm_status mm_get_diag(mm_ctx *c, mm_diag *out) {
    if (!c || !out) return MM_E_ARG;
    mm_status st0 = need_ws(c);
    if (st0 != MM_OK) return st0;
    DiagDev slots[kDiagSlots];
    int32_t nonfin = 0;
    MM_CHECK(hipMemcpyAsync(slots, c->at<char>(c->lay.diag), sizeof(slots), hipMemcpyDeviceToHost, c->st()));
    MM_CHECK(hipMemcpyAsync(&nonfin, c->at<int32_t>(c->lay.flags) + 1, sizeof(int32_t), hipMemcpyDeviceToHost,
                            c->st()));
    MM_CHECK(hipStreamSynchronize(c->st()));
    DiagDev d;
    std::memset(&d, 0, sizeof(d));
    for (int k = 0; k < kDiagSlots; k++) {
        d.newton_iters += slots[k].newton_iters;
        d.newton_max = slots[k].newton_max > d.newton_max ? slots[k].newton_max : d.newton_max;
        d.unconverged += slots[k].unconverged;
        d.vacuum += slots[k].vacuum;
        d.positivity_fallback += slots[k].positivity_fallback;
        d.fp64_fallback += slots[k].fp64_fallback;
        d.guess_fallback += slots[k].guess_fallback;
        d.wave_iter_max_sum += slots[k].wave_iter_max_sum;
        d.entropy_kept += slots[k].entropy_kept;
    }
    std::memset(out, 0, sizeof(*out));
    out->faces = c->faces_done;
    out->newton_iters = d.newton_iters;
    out->newton_max = d.newton_max;
    out->unconverged = d.unconverged;
    out->vacuum = d.vacuum;
    out->positivity_fallback = d.positivity_fallback;
    out->fp64_fallback = d.fp64_fallback;
    out->guess_fallback = d.guess_fallback;
    out->wave_iter_max_sum = d.wave_iter_max_sum;
    out->entropy_kept = d.entropy_kept;
    out->waves = c->waves_done;
    out->nonfinite = nonfin;
    return MM_OK;
}


// ------------------------------------------------------------------------
// Individual timesteps (Section 7.2).

mm_status mm_tb_begin(mm_ctx *c, double dt_max, int32_t levels) {
    if (!c) return MM_E_ARG;
    if (c->p.steps != MM_STEPS_INDIVIDUAL) return MM_E_STATE;
    if (!(dt_max > 0.0) || !isfinite(dt_max) || levels < 0 || levels > kTbMaxLevels) return MM_E_ARG;
    if (!c->have_mesh) return MM_E_STATE;
    const Layout &L = c->lay;
    // exact per-residue sums for the sparse path's sub-lists (the touched
    // list's region holds them before the timeline starts)
    int32_t *sums_dev = c->at<int32_t>(L.tb_touched);
    k_fill_i32<<<plain_grid(2 * kLists), kBlock, 0, c->st()>>>(sums_dev, 2 * kLists, 0);
    k_tb_bound<<<plain_grid(c->n), kBlock, 0, c->st()>>>(c->n, grid_for(c->n), c->at<int32_t>(L.off), sums_dev,
                                                        sums_dev + kLists);
    MM_LAUNCH_CHECK();
    int32_t sums[2 * kLists];
    MM_CHECK(hipMemcpyAsync(sums, sums_dev, sizeof(sums), hipMemcpyDeviceToHost, c->st()));
    MM_CHECK(hipStreamSynchronize(c->st()));
    int64_t ms = 0, mt = 0;
    for (int k = 0; k < kLists; k++) {
        ms = sums[k] > ms ? sums[k] : ms;
        mt = (int64_t)sums[k] + sums[kLists + k] > mt ? (int64_t)sums[k] + sums[kLists + k] : mt;
    }
    c->tb.sparse_ok = ms <= tb_face_cap(c->n, c->nf) && mt <= tb_touch_cap(c->n, c->nf);
    k_tb_init<<<plain_grid(c->n > TB_INFO_INTS ? c->n : TB_INFO_INTS), kBlock, 0, c->st()>>>(
        c->n, levels, c->at<int8_t>(L.tb_bin), c->at<int64_t>(L.tb_trec), c->at<int32_t>(L.tb_touch),
        c->at<int32_t>(L.tb_info));
    // each point's finish clears its lists for the next one; the first
    // starts from this
    k_tb_reset<<<1, kBlock, 0, c->st()>>>(c->at<int32_t>(L.tb_cells), c->at<int32_t>(L.tb_faces),
                                          c->at<int32_t>(L.tb_touched),
                                          c->p.mode == MM_MIXED ? c->at<int32_t>(L.hard) : nullptr,
                                          c->at<int32_t>(L.tb_info), c->at<int32_t>(L.flags) + 2);
    MM_LAUNCH_CHECK();
    c->tb.on = true;
    c->tb.dt_max = dt_max;
    c->tb.levels = levels;
    c->tb.ti = 0;
    return MM_OK;
}

// One synchronisation point, enqueued with the same arguments at every
// point: the tick, the path and whether the point runs at all come from the
// info block. Sparse points (at most 1/8 of the cells due) find their faces
// and touched cells from the active cells' side lists; dense points scan
// every face and update every stamped cell. Both give the same fluxes and
// sums.
template <int D, typename T> static void tb_point(mm_ctx *c, double *Q, T *rec) {
    const Layout &L = c->lay;
    hipStream_t s = c->st();
    const mm_ctx::Timeline &tb = c->tb;
    int8_t *bin = c->at<int8_t>(L.tb_bin);
    int64_t *trec = c->at<int64_t>(L.tb_trec);
    double *sig = c->at<double>(L.tb_sig);
    int32_t *touch = c->at<int32_t>(L.tb_touch);
    int32_t *cells = c->at<int32_t>(L.tb_cells), *faces = c->at<int32_t>(L.tb_faces);
    int32_t *touched = c->at<int32_t>(L.tb_touched);
    int32_t *info = c->at<int32_t>(L.tb_info);
    int32_t *flags = c->at<int32_t>(L.flags);
    const int64_t ccap = list_cap(grid_for(c->n)), fcap = tb_face_cap(c->n, c->nf);
    const int64_t tcap = tb_touch_cap(c->n, c->nf);
    const bool mixed = c->p.mode == MM_MIXED;
    const T *srec = mixed ? (const T *)c->at<float>(L.srec32) : (const T *)c->at<double>(L.srec);
    T *grad = grad_block<D>(c, rec);
    int32_t *hard = mixed ? c->at<int32_t>(L.hard) : nullptr;
    const int32_t *off = c->at<int32_t>(L.off), *ent = c->at<int32_t>(L.ent), *nbr = c->at<int32_t>(L.nbr);
    const double *w0 = mixed ? c->at<double>(L.w0) : nullptr;
    k_tb_open<D, T><<<grid_for(c->n), kBlock, 0, s>>>(c->n, info, bin, trec, c->p.gamma, c->mesh.volume, Q,
                                                      c->mesh.mesh_vel, c->mesh.centroid_off, rec, w0, sig, cells,
                                                      ccap);
    k_tb_active<D, T><<<kTbGrid, kBlock, 0, s>>>(cells, ccap, tb.dt_max, tb.levels, c->p.cfl, off, ent, nbr,
                                                 c->at<double>(L.frec), sig, bin, info, srec, c->mesh.volume, rec,
                                                 grad, touch, faces, fcap, touched, tcap);
    k_tb_faces<<<kTbGrid, kBlock, 0, s>>>(c->nf, c->mesh.face_L, c->mesh.face_R, bin, info, touch, faces, fcap);
    const TbView view{bin, trec, 0, tb.dt_max, tb.levels, info};
    DiagDev *diag = c->at<DiagDev>(L.diag);
    const MlpPacked *mlp = active_mlp(c);
    const GasConst<double> kg(c->p.gamma);
    double *flux = c->at<double>(L.flux);
    if (!mixed) {
        auto kern = mlp ? k_face_flux64_list<D, true> : k_face_flux64_list<D, false>;
        kern<<<kTbGrid, kBlock, 0, s>>>(faces, fcap, c->mesh.face_L, c->mesh.face_R, c->at<double>(L.frec),
                                        c->at<double>(L.wf64), (const double *)rec, (const double *)grad, view, kg,
                                        c->p.newton_tol64, c->p.newton_max_iter, mlp, flux, diag);
    } else {
        const GasConst<float> kf(c->p.gamma);
        auto kern = mlp ? k_face_flux_mixed_list<D, true> : k_face_flux_mixed_list<D, false>;
        kern<<<kTbGrid, kBlock, 0, s>>>(faces, fcap, c->mesh.face_L, c->mesh.face_R, c->at<float>(L.mrec),
                                        (const float *)rec, (const float *)grad, view, kf,
                                        kg.g_over_gm1, (float)c->p.newton_tol32, c->p.newton_max_iter, mlp, flux,
                                        hard, diag, face_aux(c));
        k_face_flux_hard<D, 0, false><<<kTbGrid, kBlock, 0, s>>>(
            c->mesh.face_L, c->mesh.face_R, c->at<float>(L.mrec), (const float *)rec,
            (const float *)grad, nullptr, 0.0, kf.g, kg, c->p.newton_tol64, hard, fcap, flux, diag,
            face_aux(c), view);
    }
    const TbSides sd{c->at<int32_t>(L.loff), c->at<int32_t>(L.roff), c->at<int32_t>(L.rface), c->mesh.face_L,
                     c->mesh.face_R};
    k_tb_update_list<D><<<kTbGrid, kBlock, 0, s>>>(touched, tcap, c->n, sd, bin, flux, Q, flags + 1, info);
    k_tb_update<D><<<kTbGrid, kBlock, 0, s>>>(c->n, sd, bin, info, touch, flux, Q, flags + 1);
    k_tb_finish<<<1, kBlock, 0, s>>>(c->n, tb.levels, tb.sparse_ok ? 1 : 0, cells, faces, touched, hard, flags + 2,
                                     info);
}

mm_status mm_tb_advance(mm_ctx *c, double *Q, int64_t until_tick, int32_t max_points, mm_tb_info *out) {
    if (!c || !Q || max_points < 1) return MM_E_ARG;
    if (!c->have_mesh || !c->tb.on || c->accel || c->walls.n) return MM_E_STATE;
    const Layout &L = c->lay;
    hipStream_t s = c->st();
    const bool f64 = c->p.mode == MM_FP64;
    void *rec = f64 ? (void *)c->at<double>(L.rec) : (void *)c->at<float>(L.rec32);
    int32_t *info = c->at<int32_t>(L.tb_info);
    k_tb_batch<<<1, 1, 0, s>>>(info, until_tick);
    for (int32_t k = 0; k < max_points; k++) {
        if (c->D == 3) f64 ? tb_point<3, double>(c, Q, (double *)rec) : tb_point<3, float>(c, Q, (float *)rec);
        else f64 ? tb_point<2, double>(c, Q, (double *)rec) : tb_point<2, float>(c, Q, (float *)rec);
    }
    MM_LAUNCH_CHECK();
    int32_t h[TB_INFO_INTS];
    MM_CHECK(hipMemcpyAsync(h, info, sizeof(h), hipMemcpyDeviceToHost, s));
    MM_CHECK(hipStreamSynchronize(s));
    mm_ctx::Timeline &tb = c->tb;
    auto i64 = [&](int slot) { int64_t v; std::memcpy(&v, h + slot, sizeof(v)); return v; };
    tb.ti = i64(TB_TI);
    const int64_t sumf = i64(TB_SUMF);
    c->faces_done += (uint64_t)sumf;
    c->waves_done += (uint64_t)((sumf + 63) / 64);
    if (out) {
        out->tick = i64(TB_LAST);
        out->next_tick = tb.ti;
        out->active_cells = h[TB_CELLS];
        out->active_faces = h[TB_FACES];
        out->min_bin = h[TB_LO];
        out->max_bin = h[TB_HI];
        out->sparse = h[TB_LASTSPARSE];
        out->points = h[TB_NPTS];
        out->sparse_points = h[TB_NSPARSE];
        out->total_cells = i64(TB_SUMC);
        out->total_faces = sumf;
        out->next_time = ldexp(tb.dt_max, -tb.levels) * (double)tb.ti;
    }
    if (h[TB_ERR]) {
        tb.on = false;   // bins and records of the failed point's active cells have moved on; Q has not
        return MM_E_RANGE;
    }
    return h[TB_NONFIN] ? MM_E_NONFINITE : MM_OK;
}

mm_status mm_tb_step(mm_ctx *c, double *Q, mm_tb_info *out) {
    return mm_tb_advance(c, Q, INT64_MAX, 1, out);
}

mm_status mm_tb_state(mm_ctx *c, int8_t *bins, int64_t *trec) {
    if (!c) return MM_E_ARG;
    if (!c->tb.on) return MM_E_STATE;
    const Layout &L = c->lay;
    if (bins) MM_CHECK(hipMemcpyAsync(bins, c->at<int8_t>(L.tb_bin), c->n, hipMemcpyDeviceToDevice, c->st()));
    if (trec)
        MM_CHECK(hipMemcpyAsync(trec, c->at<int64_t>(L.tb_trec), c->n * sizeof(int64_t), hipMemcpyDeviceToDevice,
                                c->st()));
    return MM_OK;
}
