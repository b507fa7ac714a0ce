// voronoi.cpp -- periodic Voronoi tessellation of a point set in the unit
// box (2D or 3D) by per-cell half-space clipping.
//
// This is an input generator: it produces the given tessellation that the
// hydro step runs on (cell volumes and centres of mass, face areas,
// centroids and generator separations). It holds none of the hydro scheme's
// arithmetic. Each cell starts as a box around its generator and is clipped
// by the bisector planes of candidate neighbours taken in order of distance;
// the search stops once every vertex of the cell lies closer than half the
// distance to the next unexamined candidate, which is the completeness test
// the paper uses for its ghost-point search (Section 2.4): a point farther
// than twice the largest vertex distance cannot cut the cell. Periodicity is
// handled by searching buckets of a wrapped grid and carrying the image
// shift into the separation vector.
//
// Output (cells in input order, faces emitted once, from the lower index):
//   volume[N], centroid_off[D][N] (s_i - r_i),
//   face_L[F] < face_R[F], face_area[F],
//   face_ctr[D][F] (f - r_L), face_sep[D][F] (r_R image - r_L).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>
#include <cstdio>

namespace {

struct V3 { double x, y, z; };
static inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
static inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
static inline V3 mul(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
static inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
static inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

struct Cand { double dist2; int64_t j; V3 d; };

struct FaceRec { int64_t nb; V3 d; double area; V3 ctr; };

// Bucket grid over the periodic unit box.
struct Grid {
    int dim; int nb; double bs; int64_t n;
    std::vector<int64_t> start, items;
    const double *pos;
    void build(const double *p, int64_t npts, int d, double target_per_bucket) {
        pos = p; n = npts; dim = d;
        double per_axis = std::pow((double)npts / target_per_bucket, 1.0 / d);
        nb = std::max(1, (int)std::floor(per_axis));
        bs = 1.0 / nb;
        int64_t nbk = 1; for (int k = 0; k < d; k++) nbk *= nb;
        std::vector<int64_t> cnt(nbk + 1, 0), key(npts);
        for (int64_t i = 0; i < npts; i++) { key[i] = bucket_of(i); cnt[key[i] + 1]++; }
        for (int64_t b = 0; b < nbk; b++) cnt[b + 1] += cnt[b];
        start = cnt; items.resize(npts);
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        for (int64_t i = 0; i < npts; i++) items[fill[key[i]]++] = i;
    }
    int cidx(double x) const { int c = (int)std::floor(x * nb); if (c < 0) c = 0; if (c >= nb) c = nb - 1; return c; }
    int64_t bucket_of(int64_t i) const {
        int64_t b = 0;
        for (int k = 0; k < dim; k++) b = b * nb + cidx(pos[i * dim + k]);
        return b;
    }
};

// Append candidates of the Chebyshev ring K around the generator's bucket.
// Distinct offsets give distinct (bucket, wrap) pairs, hence distinct
// periodic images, so K may exceed half the grid for sparse point sets.
static void gather_ring(const Grid &G, int64_t i, int K, std::vector<Cand> &out) {
    const int D = G.dim;
    int c0[3] = {0, 0, 0};
    for (int k = 0; k < D; k++) c0[k] = G.cidx(G.pos[i * D + k]);
    double ri[3] = {G.pos[i * D + 0], G.pos[i * D + 1], D == 3 ? G.pos[i * D + 2] : 0.0};
    int zlo = (D == 3) ? -K : 0, zhi = (D == 3) ? K : 0;
    for (int oz = zlo; oz <= zhi; oz++)
        for (int oy = -K; oy <= K; oy++)
            for (int ox = -K; ox <= K; ox++) {
                int m = std::max(std::abs(ox), std::max(std::abs(oy), std::abs(oz)));
                if (m != K) continue;
                int off[3] = {ox, oy, oz};
                int cb[3]; double shift[3] = {0, 0, 0};
                int64_t b = 0;
                for (int k = 0; k < D; k++) {
                    int c = c0[k] + off[k];
                    int w = (int)std::floor((double)c / G.nb);
                    cb[k] = c - w * G.nb;
                    shift[k] = (double)w;
                    b = b * G.nb + cb[k];
                }
                for (int64_t q = G.start[b]; q < G.start[b + 1]; q++) {
                    int64_t j = G.items[q];
                    if (j == i && K == 0) continue;
                    V3 d{0, 0, 0};
                    d.x = G.pos[j * D + 0] + shift[0] - ri[0];
                    d.y = G.pos[j * D + 1] + shift[1] - ri[1];
                    if (D == 3) d.z = G.pos[j * D + 2] + shift[2] - ri[2];
                    out.push_back({dot(d, d), j, d});
                }
            }
}

// ---------------------------------------------------------------- 3D cell
struct Poly3 {
    std::vector<int64_t> fnb;          // neighbour of each face (-1: initial box)
    std::vector<V3> fd;                // separation vector of each face
    std::vector<int> fstart, fcount;   // into verts
    std::vector<V3> verts;
    void clear() { fnb.clear(); fd.clear(); fstart.clear(); fcount.clear(); verts.clear(); }
};

static void init_box3(Poly3 &P, double h) {
    P.clear();
    // six faces of the cube [-h,h]^3, counter-clockwise seen from outside
    const V3 c[8] = {{-h,-h,-h},{h,-h,-h},{h,h,-h},{-h,h,-h},{-h,-h,h},{h,-h,h},{h,h,h},{-h,h,h}};
    const int F[6][4] = {{0,3,2,1},{4,5,6,7},{0,1,5,4},{2,3,7,6},{1,2,6,5},{0,4,7,3}};
    const V3 dn[6] = {{0,0,-2*h},{0,0,2*h},{0,-2*h,0},{0,2*h,0},{2*h,0,0},{-2*h,0,0}};
    for (int f = 0; f < 6; f++) {
        P.fnb.push_back(-1); P.fd.push_back(dn[f]);
        P.fstart.push_back((int)P.verts.size()); P.fcount.push_back(4);
        for (int k = 0; k < 4; k++) P.verts.push_back(c[F[f][k]]);
    }
}

static double max_r2_3(const Poly3 &P) {
    double m = 0; for (auto &v : P.verts) m = std::max(m, dot(v, v)); return m;
}

// Clip by the half-space {x : n.x <= h} with n = d/|d|, h = |d|/2.
static void clip3(const Poly3 &P, Poly3 &Q, int64_t nb, V3 d, double eps,
                  std::vector<V3> &cut, std::vector<double> &sv) {
    double ell = norm(d);
    V3 n = mul(d, 1.0 / ell);
    double h = 0.5 * ell;
    sv.resize(P.verts.size());
    bool any_out = false;
    for (size_t k = 0; k < P.verts.size(); k++) { sv[k] = dot(n, P.verts[k]) - h; if (sv[k] > eps) any_out = true; }
    if (!any_out) { Q = P; return; }
    Q.clear(); cut.clear();
    for (size_t f = 0; f < P.fnb.size(); f++) {
        int s0 = P.fstart[f], m = P.fcount[f];
        int qs = (int)Q.verts.size();
        for (int a = 0; a < m; a++) {
            int b = (a + 1) % m;
            double sa = sv[s0 + a], sb = sv[s0 + b];
            const V3 &va = P.verts[s0 + a], &vb = P.verts[s0 + b];
            bool ina = sa <= eps, inb = sb <= eps;
            if (ina) {
                Q.verts.push_back(va);
                if (sa >= -eps) cut.push_back(va);
            }
            if (ina != inb) {
                // one strictly outside: intersection with the plane
                double t = sa / (sa - sb);
                V3 p = add(va, mul(sub(vb, va), t));
                if (!(ina && sa >= -eps) && !(inb && sb >= -eps)) {
                    Q.verts.push_back(p);
                    cut.push_back(p);
                } else if (!ina) {
                    // b is on the plane and will be emitted as b itself
                }
            }
        }
        int cnt = (int)Q.verts.size() - qs;
        if (cnt >= 3) {
            Q.fnb.push_back(P.fnb[f]); Q.fd.push_back(P.fd[f]);
            Q.fstart.push_back(qs); Q.fcount.push_back(cnt);
        } else {
            Q.verts.resize(qs);
        }
    }
    // new face from the cut points, ordered by angle around their mean
    if (cut.size() >= 3) {
        V3 mean{0, 0, 0};
        for (auto &p : cut) mean = add(mean, p);
        mean = mul(mean, 1.0 / cut.size());
        V3 u = (std::fabs(n.x) < 0.9) ? V3{1, 0, 0} : V3{0, 1, 0};
        u = sub(u, mul(n, dot(u, n))); u = mul(u, 1.0 / norm(u));
        V3 v = cross(n, u);
        std::vector<std::pair<double, V3>> ang;
        ang.reserve(cut.size());
        for (auto &p : cut) { V3 q = sub(p, mean); ang.push_back({std::atan2(dot(q, v), dot(q, u)), p}); }
        std::sort(ang.begin(), ang.end(), [](const std::pair<double, V3> &a, const std::pair<double, V3> &b) { return a.first < b.first; });
        int qs = (int)Q.verts.size();
        for (auto &a : ang) {
            if ((int)Q.verts.size() > qs) {
                V3 last = Q.verts.back();
                if (norm(sub(last, a.second)) <= 4 * eps) continue;
            }
            Q.verts.push_back(a.second);
        }
        while ((int)Q.verts.size() - qs >= 2 && norm(sub(Q.verts.back(), Q.verts[qs])) <= 4 * eps) Q.verts.pop_back();
        int cnt = (int)Q.verts.size() - qs;
        if (cnt >= 3) {
            Q.fnb.push_back(nb); Q.fd.push_back(d);
            Q.fstart.push_back(qs); Q.fcount.push_back(cnt);
        } else {
            Q.verts.resize(qs);
        }
    }
}

struct CellOut { double vol; V3 cen; std::vector<FaceRec> faces; int status; };

static void build_cell3(const Grid &G, int64_t i, Poly3 &A, Poly3 &B, std::vector<Cand> &cands,
                        std::vector<V3> &cut, std::vector<double> &sv, CellOut &out) {
    init_box3(A, 0.5);
    cands.clear();
    int K = 0;
    gather_ring(G, i, 0, cands);
    K = 1; gather_ring(G, i, 1, cands);
    std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.dist2 < b.dist2 || (a.dist2 == b.dist2 && a.j < b.j); });
    size_t idx = 0;
    Poly3 *P = &A, *Q = &B;
    double r2max = max_r2_3(*P);
    int maxK = 4 * G.nb;  // distinct ring offsets always give distinct periodic images
    out.status = 0;
    while (true) {
        double covered = K * G.bs;
        bool done = false;
        while (idx < cands.size()) {
            const Cand &c = cands[idx];
            // only a candidate inside the gathered radius is known to be the
            // nearest unexamined point; beyond it the next ring may hold
            // nearer ones
            if (c.dist2 >= covered * covered) break;
            if (c.dist2 > 4.0 * r2max) { done = true; break; }
            double eps = 1e-12 * std::sqrt(r2max);
            clip3(*P, *Q, c.j, c.d, eps, cut, sv);
            std::swap(P, Q);
            r2max = max_r2_3(*P);
            idx++;
        }
        if (done || 4.0 * r2max <= covered * covered) break;
        if (K + 1 > maxK) { out.status = 1; break; }
        K++;
        size_t old = cands.size();
        gather_ring(G, i, K, cands);
        std::sort(cands.begin() + idx, cands.end(), [](const Cand &a, const Cand &b) { return a.dist2 < b.dist2 || (a.dist2 == b.dist2 && a.j < b.j); });
        (void)old;
    }
    // geometry
    out.faces.clear();
    double vol = 0; V3 cen{0, 0, 0};
    for (size_t f = 0; f < P->fnb.size(); f++) {
        if (P->fnb[f] < 0) { out.status = 2; continue; }
        int s0 = P->fstart[f], m = P->fcount[f];
        V3 v0 = P->verts[s0];
        double area = 0; V3 fc{0, 0, 0};
        V3 n = mul(P->fd[f], 1.0 / norm(P->fd[f]));
        for (int k = 1; k + 1 < m; k++) {
            V3 a = sub(P->verts[s0 + k], v0), b = sub(P->verts[s0 + k + 1], v0);
            double ta = 0.5 * dot(cross(a, b), n);
            area += ta;
            fc = add(fc, mul(add(add(v0, P->verts[s0 + k]), P->verts[s0 + k + 1]), ta / 3.0));
        }
        if (area < 0) { area = -area; fc = mul(fc, -1.0); }
        if (area <= 0) continue;
        fc = mul(fc, 1.0 / area);
        double hgt = 0.5 * norm(P->fd[f]);
        double pv = area * hgt / 3.0;
        vol += pv;
        cen = add(cen, mul(fc, 0.75 * pv));
        out.faces.push_back({P->fnb[f], P->fd[f], area, fc});
    }
    out.vol = vol;
    out.cen = mul(cen, 1.0 / vol);
    std::sort(out.faces.begin(), out.faces.end(), [](const FaceRec &a, const FaceRec &b) { return a.nb < b.nb; });
}

// ---------------------------------------------------------------- 2D cell
struct Poly2 { std::vector<V3> v; std::vector<int64_t> enb; std::vector<V3> ed; };

static void clip2(const Poly2 &P, Poly2 &Q, int64_t nb, V3 d, double eps) {
    double ell = norm(d);
    V3 n = mul(d, 1.0 / ell);
    double h = 0.5 * ell;
    size_t m = P.v.size();
    bool any_out = false;
    std::vector<double> s(m);
    for (size_t k = 0; k < m; k++) { s[k] = dot(n, P.v[k]) - h; if (s[k] > eps) any_out = true; }
    if (!any_out) { Q = P; return; }
    Q.v.clear(); Q.enb.clear(); Q.ed.clear();
    // edge k runs from v[k] to v[k+1] and carries label enb[k]
    for (size_t a = 0; a < m; a++) {
        size_t b = (a + 1) % m;
        bool ina = s[a] <= eps, inb = s[b] <= eps;
        if (ina) {
            Q.v.push_back(P.v[a]);
            if (inb) { Q.enb.push_back(P.enb[a]); Q.ed.push_back(P.ed[a]); }
            else {
                // leaving: the kept part of this edge, then the new edge
                double t = s[a] / (s[a] - s[b]);
                V3 p = add(P.v[a], mul(sub(P.v[b], P.v[a]), t));
                if (s[a] >= -eps) {
                    // a itself lies on the cutting line: new edge starts at a
                    Q.enb.push_back(nb); Q.ed.push_back(d);
                } else {
                    Q.enb.push_back(P.enb[a]); Q.ed.push_back(P.ed[a]);
                    Q.v.push_back(p); Q.enb.push_back(nb); Q.ed.push_back(d);
                }
            }
        } else if (inb) {
            // entering: the intersection starts the rest of edge a
            if (s[b] >= -eps) continue;
            double t = s[a] / (s[a] - s[b]);
            V3 p = add(P.v[a], mul(sub(P.v[b], P.v[a]), t));
            Q.v.push_back(p); Q.enb.push_back(P.enb[a]); Q.ed.push_back(P.ed[a]);
        }
    }
    // drop zero-length edges
    Poly2 R;
    size_t q = Q.v.size();
    for (size_t k = 0; k < q; k++) {
        V3 a = Q.v[k], b = Q.v[(k + 1) % q];
        if (norm(sub(b, a)) <= 4 * eps) continue;
        R.v.push_back(a); R.enb.push_back(Q.enb[k]); R.ed.push_back(Q.ed[k]);
    }
    Q = R;
}

static void build_cell2(const Grid &G, int64_t i, std::vector<Cand> &cands, CellOut &out) {
    Poly2 P, Q;
    const double h = 0.5;
    P.v = {{-h, -h, 0}, {h, -h, 0}, {h, h, 0}, {-h, h, 0}};
    P.enb = {-1, -1, -1, -1};
    P.ed = {{0, -2 * h, 0}, {2 * h, 0, 0}, {0, 2 * h, 0}, {-2 * h, 0, 0}};
    cands.clear();
    gather_ring(G, i, 0, cands);
    int K = 1; gather_ring(G, i, 1, cands);
    auto cmp = [](const Cand &a, const Cand &b) { return a.dist2 < b.dist2 || (a.dist2 == b.dist2 && a.j < b.j); };
    std::sort(cands.begin(), cands.end(), cmp);
    size_t idx = 0;
    auto r2 = [&]() { double m = 0; for (auto &v : P.v) m = std::max(m, dot(v, v)); return m; };
    double r2max = r2();
    int maxK = 4 * G.nb;  // distinct ring offsets always give distinct periodic images
    out.status = 0;
    while (true) {
        double covered = K * G.bs;
        bool done = false;
        while (idx < cands.size()) {
            const Cand &c = cands[idx];
            if (c.dist2 >= covered * covered) break;   // as in 3D
            if (c.dist2 > 4.0 * r2max) { done = true; break; }
            clip2(P, Q, c.j, c.d, 1e-12 * std::sqrt(r2max));
            std::swap(P, Q);
            r2max = r2();
            idx++;
        }
        if (done || 4.0 * r2max <= covered * covered) break;
        if (K + 1 > maxK) { out.status = 1; break; }
        K++;
        gather_ring(G, i, K, cands);
        std::sort(cands.begin() + idx, cands.end(), cmp);
    }
    out.faces.clear();
    double vol = 0; V3 cen{0, 0, 0};
    size_t m = P.v.size();
    for (size_t k = 0; k < m; k++) {
        V3 a = P.v[k], b = P.v[(k + 1) % m];
        double tri = 0.5 * (a.x * b.y - a.y * b.x);
        vol += tri;
        cen = add(cen, mul(add(a, b), tri / 3.0));
        if (P.enb[k] < 0) { out.status = 2; continue; }
        double len = norm(sub(b, a));
        if (len <= 0) continue;
        out.faces.push_back({P.enb[k], P.ed[k], len, mul(add(a, b), 0.5)});
    }
    out.vol = vol;
    out.cen = mul(cen, 1.0 / vol);
    std::sort(out.faces.begin(), out.faces.end(), [](const FaceRec &a, const FaceRec &b) { return a.nb < b.nb; });
}

struct Result {
    int dim; int64_t n, nf; int64_t n_bad, n_asym;
    std::vector<double> vol, coff;
    std::vector<int32_t> L, R;
    std::vector<double> area, ctr, sep;
};

}  // namespace

extern "C" {

// Build the tessellation. pos is [n][dim] in [0,1). Returns an opaque
// handle (NULL on allocation failure); query sizes with vor_counts.
void *vor_build(int32_t dim, int64_t n, const double *pos, int32_t nthreads) {
    if ((dim != 2 && dim != 3) || n < 2) return nullptr;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    Grid G; G.build(pos, n, dim, 2.0);
    std::vector<CellOut> cells(n);
    std::atomic<int64_t> bad{0}, done{0};
    // large builds (minutes) report each tenth of the cells on stderr
    const bool report = n >= (int64_t(1) << 22);
#pragma omp parallel
    {
        Poly3 A, B; std::vector<Cand> cands; std::vector<V3> cut; std::vector<double> sv;
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; i++) {
            if (dim == 3) build_cell3(G, i, A, B, cands, cut, sv, cells[i]);
            else build_cell2(G, i, cands, cells[i]);
            if (cells[i].status) bad++;
            if (report) {
                const int64_t d = ++done;
                if (d % ((n + 9) / 10) == 0) {
                    fprintf(stderr, "voronoi: %lld of %lld cells\n", (long long)d, (long long)n);
                    fflush(stderr);
                }
            }
        }
    }
    Result *res = new Result();
    res->dim = dim; res->n = n; res->n_bad = bad.load();
    res->vol.resize(n); res->coff.resize((size_t)dim * n);
    std::vector<int64_t> off(n + 1, 0);
    for (int64_t i = 0; i < n; i++) {
        int64_t c = 0;
        for (auto &f : cells[i].faces) if (f.nb > i) c++;
        off[i + 1] = off[i] + c;
    }
    int64_t nf = off[n];
    res->nf = nf;
    res->L.resize(nf); res->R.resize(nf); res->area.resize(nf);
    res->ctr.resize((size_t)dim * nf); res->sep.resize((size_t)dim * nf);
    // asymmetry: a face listed by one side only
    std::atomic<int64_t> asym{0};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const CellOut &c = cells[i];
        res->vol[i] = c.vol;
        res->coff[0 * n + i] = c.cen.x;
        res->coff[1 * n + i] = c.cen.y;
        if (dim == 3) res->coff[2 * n + i] = c.cen.z;
        int64_t o = off[i];
        for (auto &f : c.faces) {
            const auto &nf2 = cells[f.nb].faces;
            bool found = std::binary_search(nf2.begin(), nf2.end(), FaceRec{i, {0, 0, 0}, 0, {0, 0, 0}},
                                            [](const FaceRec &a, const FaceRec &b) { return a.nb < b.nb; });
            if (!found) asym++;
            if (f.nb <= i) continue;
            res->L[o] = (int32_t)i; res->R[o] = (int32_t)f.nb;
            res->area[o] = f.area;
            res->ctr[0 * nf + o] = f.ctr.x; res->ctr[1 * nf + o] = f.ctr.y;
            res->sep[0 * nf + o] = f.d.x; res->sep[1 * nf + o] = f.d.y;
            if (dim == 3) { res->ctr[2 * nf + o] = f.ctr.z; res->sep[2 * nf + o] = f.d.z; }
            o++;
        }
    }
    res->n_asym = asym.load();
    return res;
}

// counts[0] = faces, counts[1] = cells whose search failed or stayed open,
// counts[2] = face listings seen from one side only.
void vor_counts(void *h, int64_t *counts) {
    Result *r = (Result *)h;
    counts[0] = r->nf; counts[1] = r->n_bad; counts[2] = r->n_asym;
}

void vor_fetch(void *h, double *volume, double *centroid_off, int32_t *L, int32_t *R,
               double *area, double *ctr, double *sep) {
    Result *r = (Result *)h;
    std::memcpy(volume, r->vol.data(), sizeof(double) * r->n);
    std::memcpy(centroid_off, r->coff.data(), sizeof(double) * r->dim * r->n);
    std::memcpy(L, r->L.data(), sizeof(int32_t) * r->nf);
    std::memcpy(R, r->R.data(), sizeof(int32_t) * r->nf);
    std::memcpy(area, r->area.data(), sizeof(double) * r->nf);
    std::memcpy(ctr, r->ctr.data(), sizeof(double) * r->dim * r->nf);
    std::memcpy(sep, r->sep.data(), sizeof(double) * r->dim * r->nf);
}

void vor_free(void *h) { delete (Result *)h; }

}  // extern "C"
