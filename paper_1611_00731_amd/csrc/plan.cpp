// Host planner of the PUFE assembly: DOF map, enriched sets, block layout,
// element tables and colouring.  Runs once per geometry, before any device
// work (the paper builds one quadrature rule and one basis per geometry and
// reuses them for every integral, section "Adaptive quadrature").
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <array>
#include <map>
#include <set>
#include <tuple>

namespace pufe {

namespace {

// The C^3 cutoff of section "Partition of unity enrichment functions",
// h(r, rc) = 1 - 35 x^4 + 84 x^5 - 70 x^6 + 20 x^7 with x = r/rc (r <= rc).
double cutoff_h(double r, double rc) {
    const double x = std::min(r / rc, 1.0), x4 = (x * x) * (x * x);
    return 1.0 + x4 * (-35.0 + x * (84.0 + x * (-70.0 + 20.0 * x)));
}

// Clamped cubic spline through y_j = t_j h(r_j, rc), r_j = j dr, with zero end
// slopes, as C^2 Hermite pieces: the knot slopes s_j solve
//   s_{j-1} + 4 s_j + s_{j+1} = 3 (y_{j+1} - y_{j-1}) / dr   (0 < j < n-1),
// s_0 = s_{n-1} = 0; piece j in powers of tau = (r - r_j) / dr:
//   y_j + (s_j dr) tau + (3 dy - (2 s_j + s_{j+1}) dr) tau^2
//       + ((s_j + s_{j+1}) dr - 2 dy) tau^3,   dy = y_{j+1} - y_j.
void radial_spline(const std::vector<double> &t, double rc, std::vector<double> &out) {
    const int n = (int)t.size();
    const double dr = rc / (n - 1);
    std::vector<double> y(n), sl(n, 0.0);
    for (int j = 0; j < n; ++j) y[j] = t[j] * cutoff_h(j * dr, rc);
    // interior slopes: tridiagonal (1, 4, 1) system, eliminated downwards
    const int m = n - 2;
    std::vector<double> cp(std::max(m, 1)), dp(std::max(m, 1));
    for (int i = 0; i < m; ++i) {
        const int j = i + 1;
        const double rhs = 3.0 * (y[j + 1] - y[j - 1]) / dr;
        const double den = 4.0 - (i > 0 ? cp[i - 1] : 0.0);
        cp[i] = 1.0 / den;
        dp[i] = (rhs - (i > 0 ? dp[i - 1] : 0.0)) / den;
    }
    for (int i = m - 1; i >= 0; --i) sl[i + 1] = dp[i] - (i + 1 < m ? cp[i] * sl[i + 2] : 0.0);
    for (int j = 0; j + 1 < n; ++j) {
        const double dy = y[j + 1] - y[j];
        out.push_back(y[j]);
        out.push_back(sl[j] * dr);
        out.push_back(3.0 * dy - (2.0 * sl[j] + sl[j + 1]) * dr);
        out.push_back((sl[j] + sl[j + 1]) * dr - 2.0 * dy);
    }
}

double det3(const double *m) {
    return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
           m[2] * (m[3] * m[7] - m[4] * m[6]);
}

// Inverse of the matrix whose rows are a_1..a_3; column d of it is the dual
// vector a*_d with a*_d . a_e = delta_de.
void inverse3(const double *m, double *o) {
    double d = det3(m);
    o[0] = (m[4] * m[8] - m[5] * m[7]) / d;
    o[1] = (m[2] * m[7] - m[1] * m[8]) / d;
    o[2] = (m[1] * m[5] - m[2] * m[4]) / d;
    o[3] = (m[5] * m[6] - m[3] * m[8]) / d;
    o[4] = (m[0] * m[8] - m[2] * m[6]) / d;
    o[5] = (m[2] * m[3] - m[0] * m[5]) / d;
    o[6] = (m[3] * m[7] - m[4] * m[6]) / d;
    o[7] = (m[1] * m[6] - m[0] * m[7]) / d;
    o[8] = (m[0] * m[4] - m[1] * m[3]) / d;
}

inline int wrapi(int j, int n) { return ((j % n) + n) % n; }

}  // namespace

int build_plan(const Problem &pr, Plan &pl, std::string &err) {
    const int n1 = pr.mesh[0], n2 = pr.mesh[1], n3 = pr.mesh[2];
    if (n1 < 2 || n2 < 2 || n3 < 2) { err = "every mesh dimension must be >= 2"; return PUFE_ERR_INVALID_ARG; }
    if (pr.p < 1 || pr.p > 3) { err = "fe_order must be 1, 2 or 3 (32-node serendipity)"; return PUFE_ERR_INVALID_ARG; }
    std::memcpy(pl.lat, pr.lat, sizeof pl.lat);
    pl.vol = det3(pr.lat);
    if (!(pl.vol > 0)) { err = "lattice must be right-handed with positive volume"; return PUFE_ERR_INVALID_ARG; }
    inverse3(pr.lat, pl.inv);
    const int n_atoms = (int)pr.species.size();
    int max_species = -1;
    for (int s : pr.species) max_species = std::max(max_species, s);
    for (const auto &e : pr.enr) {
        if (e.l < 0 || e.l > 3) { err = "enrichment l must be in 0..3"; return PUFE_ERR_INVALID_ARG; }
        if (e.radial_kind != 0 && e.radial_kind != 1) { err = "radial_kind must be 0 or 1"; return PUFE_ERR_INVALID_ARG; }
        if (!(e.rc > 0) || !(e.re >= 0) || (e.radial_kind == 0 && !(e.a > 0))) {
            err = "enrichment needs rc > 0, re >= 0 and (analytic radial) a > 0";
            return PUFE_ERR_INVALID_ARG;
        }
    }
    if (pr.radial.size() != pr.enr.size()) { err = "radial tables do not match the descriptors"; return PUFE_ERR_INVALID_ARG; }
    for (size_t k = 0; k < pr.enr.size(); ++k) {
        const auto &t = pr.radial[k];
        if (pr.enr[k].radial_kind == 0 ? !t.empty() : (t.size() < 4 || t.size() > 4096)) {
            err = "a tabulated radial needs 4..4096 samples (none for the analytic kind)";
            return PUFE_ERR_INVALID_ARG;
        }
        for (double v : t)
            if (!std::isfinite(v)) { err = "radial samples must be finite"; return PUFE_ERR_INVALID_ARG; }
    }
    for (const auto &pj : pr.proj) {
        if (pj.l < 0 || pj.l > 3) { err = "projector l must be in 0..3"; return PUFE_ERR_INVALID_ARG; }
        if (!(pj.a > 0) || !(pj.rc > 0) || !std::isfinite(pj.h)) { err = "projector needs a > 0, rc > 0, finite h"; return PUFE_ERR_INVALID_ARG; }
    }
    if (pr.enr_phase != PUFE_ENR_PERIODIC && pr.enr_phase != PUFE_ENR_BLOCH) {
        err = "unknown enrichment phase form"; return PUFE_ERR_INVALID_ARG;
    }
    const pufe_quad &q = pr.quad;
    if (q.n_gauss < 1 || q.n_gauss > kMaxGauss) { err = "n_gauss must be in 1..12"; return PUFE_ERR_INVALID_ARG; }
    if (q.max_level < 0 || q.max_level > kMaxLevel) { err = "max_level must be in 0..8"; return PUFE_ERR_INVALID_ARG; }
    if (q.mode != PUFE_QUAD_GEOM && q.mode != PUFE_QUAD_ERROR) { err = "unknown quadrature mode"; return PUFE_ERR_INVALID_ARG; }
    if (q.mode == PUFE_QUAD_ERROR && (q.n_ref <= q.n_gauss || q.n_ref > kMaxGauss)) {
        err = "error mode needs n_gauss < n_ref <= 12"; return PUFE_ERR_INVALID_ARG;
    }
    bool ortho = pr.lat[1] == 0 && pr.lat[2] == 0 && pr.lat[3] == 0 && pr.lat[5] == 0 && pr.lat[6] == 0 && pr.lat[7] == 0;
    if (q.mode == PUFE_QUAD_GEOM && q.max_level > 0 && !ortho) {
        err = "geometric refinement needs an orthorhombic cell"; return PUFE_ERR_UNSUPPORTED;
    }

    pl.nel = (int64_t)n1 * n2 * n3;
    pl.nv = pl.nel;
    // FE slots per vertex: the vertex node; triquadratic also the midpoints
    // of its 3 positive edges, 3 positive faces and its cell (8 in all);
    // serendipity also the 2 nodes of each of its 3 positive edges (7)
    pl.nfs = pr.p == 1 ? 1 : (pr.p == 2 ? 8 : 7);
    pl.nfe = pr.p == 1 ? 8 : (pr.p == 2 ? 27 : 32);
    const int mesh[3] = {n1, n2, n3};

    // ---- enriched sets: for every atom image, the vertices inside its
    // support sphere (strictly closer than re) carry the descriptor
    // (section "Partition of unity enrichment functions").
    std::vector<std::set<std::pair<int, int>>> carry(pl.nv);  // (atom, desc)
    for (int A = 0; A < n_atoms; ++A) {
        const double *tau = &pr.pos[3 * A];
        double tr[3];
        for (int d = 0; d < 3; ++d) tr[d] = tau[0] * pl.inv[0 * 3 + d] + tau[1] * pl.inv[1 * 3 + d] + tau[2] * pl.inv[2 * 3 + d];
        for (int k = 0; k < (int)pr.enr.size(); ++k) {
            if (pr.enr[k].species != pr.species[A]) continue;
            double re = pr.enr[k].re;
            if (re <= 0) continue;
            double rad[3];
            for (int d = 0; d < 3; ++d)
                rad[d] = re * std::sqrt(pl.inv[d] * pl.inv[d] + pl.inv[3 + d] * pl.inv[3 + d] + pl.inv[6 + d] * pl.inv[6 + d]);
            // vertex grid indices j (unwrapped) with |x(j) - tau| < re
            int lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
                lo[d] = (int)std::floor((tr[d] - rad[d]) * mesh[d]) - 1;
                hi[d] = (int)std::ceil((tr[d] + rad[d]) * mesh[d]) + 1;
            }
            for (int j3 = lo[2]; j3 <= hi[2]; ++j3)
                for (int j2 = lo[1]; j2 <= hi[1]; ++j2)
                    for (int j1 = lo[0]; j1 <= hi[0]; ++j1) {
                        double u[3] = {(double)j1 / n1, (double)j2 / n2, (double)j3 / n3};
                        double dx[3];
                        for (int c = 0; c < 3; ++c)
                            dx[c] = u[0] * pr.lat[c] + u[1] * pr.lat[3 + c] + u[2] * pr.lat[6 + c] - tau[c];
                        double r2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
                        if (!(std::sqrt(r2) < re)) continue;
                        int64_t v = ((int64_t)wrapi(j3, n3) * n2 + wrapi(j2, n2)) * n1 + wrapi(j1, n1);
                        carry[v].insert({A, k});
                    }
        }
    }
    pl.vf_off.assign(pl.nv + 1, 0);
    pl.vf.clear();
    for (int64_t v = 0; v < pl.nv; ++v) {
        pl.vf_off[v] = (int64_t)pl.vf.size() / 3;
        for (auto &ak : carry[v]) {  // std::set order: atom, then descriptor
            int l = pr.enr[ak.second].l;
            for (int m = -l; m <= l; ++m) {
                pl.vf.push_back(ak.first);
                pl.vf.push_back(ak.second);
                pl.vf.push_back(m);
            }
        }
    }
    pl.vf_off[pl.nv] = (int64_t)pl.vf.size() / 3;
    pl.dof_off.assign(pl.nv + 1, 0);
    for (int64_t v = 0; v < pl.nv; ++v)
        pl.dof_off[v + 1] = pl.dof_off[v] + pl.nfs + (pl.vf_off[v + 1] - pl.vf_off[v]);

    // ---- element geometry
    const double lat[9] = {pr.lat[0], pr.lat[1], pr.lat[2], pr.lat[3], pr.lat[4], pr.lat[5], pr.lat[6], pr.lat[7], pr.lat[8]};
    double E[9];
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) E[3 * d + c] = lat[3 * d + c] / mesh[d];
    // bounding radius of one element: half its longest diagonal
    double Re = 0;
    for (int s2 = -1; s2 <= 1; s2 += 2)
        for (int s3 = -1; s3 <= 1; s3 += 2) {
            double dd[3];
            for (int c = 0; c < 3; ++c) dd[c] = E[c] + s2 * E[3 + c] + s3 * E[6 + c];
            Re = std::max(Re, 0.5 * std::sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]));
        }
    auto elem_centre = [&](int64_t e, double *centre) {
        const int i0 = (int)(e % n1), i1 = (int)((e / n1) % n2), i2 = (int)(e / ((int64_t)n1 * n2));
        for (int c = 0; c < 3; ++c) centre[c] = (i0 + 0.5) * E[c] + (i1 + 0.5) * E[3 + c] + (i2 + 0.5) * E[6 + c];
    };
    auto corner_vertex = [&](int64_t e, int c) -> int64_t {
        const int i[3] = {(int)(e % n1), (int)((e / n1) % n2), (int)(e / ((int64_t)n1 * n2))};
        int j[3];
        for (int d = 0; d < 3; ++d) j[d] = (i[d] + ((c >> d) & 1)) % mesh[d];
        return ((int64_t)j[2] * n2 + j[1]) * n1 + j[0];
    };

    // ---- separable nonlocal term: projector functions J = (descriptor,
    // atom of its species, m) in that order, the projector images that
    // reach each element (sphere of radius rc around the image within the
    // element's bounding sphere), and the vertices each atom couples: a
    // projector function is the Bloch sum over all images of its atom, so
    // two vertices that reach different images of one atom are coupled too
    struct PImg {
        int A, d, n[3];
        double C[3];
    };
    std::vector<std::vector<PImg>> elem_pimg(pl.nel);
    std::vector<std::vector<int64_t>> atom_vertices(n_atoms);   // vertices of elements an image of the atom reaches
    std::vector<std::vector<int>> pfun_of(pr.proj.size(), std::vector<int>(n_atoms, -1));   // J of (d, A, m = -l)
    pl.n_pfun = 0;
    pl.pfun_h.clear();
    for (size_t d = 0; d < pr.proj.size(); ++d)
        for (int A = 0; A < n_atoms; ++A)
            if (pr.species[A] == pr.proj[d].species) {
                pfun_of[d][A] = pl.n_pfun;
                for (int m = -pr.proj[d].l; m <= pr.proj[d].l; ++m) pl.pfun_h.push_back(pr.proj[d].h);
                pl.n_pfun += 2 * pr.proj[d].l + 1;
            }
    for (int64_t e = 0; e < pl.nel && !pr.proj.empty(); ++e) {
        double centre[3], uc[3];
        elem_centre(e, centre);
        for (int d = 0; d < 3; ++d) uc[d] = centre[0] * pl.inv[d] + centre[1] * pl.inv[3 + d] + centre[2] * pl.inv[6 + d];
        for (size_t dp = 0; dp < pr.proj.size(); ++dp)
            for (int A = 0; A < n_atoms; ++A) {
                if (pr.species[A] != pr.proj[dp].species) continue;
                const double *tau = &pr.pos[3 * A];
                double ur[3];
                for (int d = 0; d < 3; ++d) ur[d] = tau[0] * pl.inv[d] + tau[1] * pl.inv[3 + d] + tau[2] * pl.inv[6 + d];
                const double reach = pr.proj[dp].rc + Re;
                int lo[3], hi[3];
                for (int d = 0; d < 3; ++d) {
                    double rad = reach * std::sqrt(pl.inv[d] * pl.inv[d] + pl.inv[3 + d] * pl.inv[3 + d] + pl.inv[6 + d] * pl.inv[6 + d]);
                    lo[d] = (int)std::floor(uc[d] - ur[d] - rad) - 1;
                    hi[d] = (int)std::ceil(uc[d] - ur[d] + rad) + 1;
                }
                for (int m3 = lo[2]; m3 <= hi[2]; ++m3)
                    for (int m2 = lo[1]; m2 <= hi[1]; ++m2)
                        for (int m1 = lo[0]; m1 <= hi[0]; ++m1) {
                            PImg pi{A, (int)dp, {m1, m2, m3}, {0, 0, 0}};
                            for (int c = 0; c < 3; ++c) pi.C[c] = tau[c] + m1 * lat[c] + m2 * lat[3 + c] + m3 * lat[6 + c];
                            const double dx = pi.C[0] - centre[0], dy = pi.C[1] - centre[1], dz = pi.C[2] - centre[2];
                            if (std::sqrt(dx * dx + dy * dy + dz * dz) >= reach) continue;
                            elem_pimg[e].push_back(pi);
                            for (int c = 0; c < 8; ++c) atom_vertices[A].push_back(corner_vertex(e, c));
                        }
            }
    }
    std::vector<std::vector<int64_t>> extra(pr.proj.empty() ? 0 : pl.nv);
    for (auto &vs : atom_vertices) {
        std::sort(vs.begin(), vs.end());
        vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
        for (int64_t v : vs) extra[v].insert(extra[v].end(), vs.begin(), vs.end());
    }

    // ---- block layout: vertex v couples to every vertex of the elements
    // around it, i.e. its (wrapped) 3x3x3 neighbourhood, and to the vertices
    // that reach a projector image with it
    auto vid = [&](int j1, int j2, int j3) -> int64_t {
        return ((int64_t)wrapi(j3, n3) * n2 + wrapi(j2, n2)) * n1 + wrapi(j1, n1);
    };
    pl.brow_ptr.assign(pl.nv + 1, 0);
    pl.bcol.clear();
    pl.brow.clear();
    pl.bval_off.clear();
    int64_t val = 0;
    for (int64_t v = 0; v < pl.nv; ++v) {
        pl.brow_ptr[v] = (int64_t)pl.bcol.size();
        int j1 = (int)(v % n1), j2 = (int)((v / n1) % n2), j3 = (int)(v / ((int64_t)n1 * n2));
        std::vector<int64_t> nb;
        for (int d3 = -1; d3 <= 1; ++d3)
            for (int d2 = -1; d2 <= 1; ++d2)
                for (int d1 = -1; d1 <= 1; ++d1) nb.push_back(vid(j1 + d1, j2 + d2, j3 + d3));
        if (!extra.empty()) nb.insert(nb.end(), extra[v].begin(), extra[v].end());
        std::sort(nb.begin(), nb.end());
        nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        int64_t bv = pl.dof_off[v + 1] - pl.dof_off[v];
        for (int64_t w : nb) {
            pl.bcol.push_back((int32_t)w);
            pl.brow.push_back((int32_t)v);
            pl.bval_off.push_back(val);
            val += bv * (pl.dof_off[w + 1] - pl.dof_off[w]);
        }
    }
    pl.brow_ptr[pl.nv] = (int64_t)pl.bcol.size();
    pl.bval_off.push_back(val);
    pl.nnz = val;
    auto block_of = [&](int64_t v, int64_t w) -> int64_t {
        auto b = pl.bcol.begin() + pl.brow_ptr[v], e = pl.bcol.begin() + pl.brow_ptr[v + 1];
        auto it = std::lower_bound(b, e, (int32_t)w);
        return pl.bval_off[it - pl.bcol.begin()];
    };
    // the blocks a projector function couples
    pl.nl_blocks.clear();
    for (const auto &vs : atom_vertices)
        for (int64_t v : vs)
            for (int64_t w : vs) {
                auto b = pl.bcol.begin() + pl.brow_ptr[v], e = pl.bcol.begin() + pl.brow_ptr[v + 1];
                pl.nl_blocks.push_back((int32_t)(std::lower_bound(b, e, (int32_t)w) - pl.bcol.begin()));
            }
    std::sort(pl.nl_blocks.begin(), pl.nl_blocks.end());
    pl.nl_blocks.erase(std::unique(pl.nl_blocks.begin(), pl.nl_blocks.end()), pl.nl_blocks.end());

    // ---- elements
    pl.elems.assign(pl.nel, ElemDev{});
    pl.pgroups.clear();
    pl.max_ncol = pl.max_npg = 0;
    pl.groups.clear();
    pl.img.clear();
    pl.img_nk.clear();
    pl.edof.clear();
    pl.bpart.clear();
    pl.bloch = pr.enr_phase == PUFE_ENR_BLOCH;
    pl.max_nloc = pl.max_nfun = pl.max_ngrp = 0;
    pl.max_l = 0;
    pl.max_img = 0;
    for (const auto &en : pr.enr) pl.max_l = std::max(pl.max_l, en.l);
    pl.spl.clear();
    pl.spl_off.assign(pr.enr.size(), -1);
    for (size_t k = 0; k < pr.enr.size(); ++k)
        if (pr.enr[k].radial_kind == 1) {
            pl.spl_off[k] = (int32_t)pl.spl.size();
            radial_spline(pr.radial[k], pr.enr[k].rc, pl.spl);
        }
    std::vector<std::vector<int32_t>> by_color(27);
    for (int64_t e = 0; e < pl.nel; ++e) {
        ElemDev &el = pl.elems[e];
        int i[3] = {(int)(e % n1), (int)((e / n1) % n2), (int)(e / ((int64_t)n1 * n2))};
        for (int d = 0; d < 3; ++d) el.ijk[d] = i[d];
        int64_t cv[8];
        el.shifts = 0;
        for (int c = 0; c < 8; ++c) {
            int j[3];
            for (int d = 0; d < 3; ++d) {
                int b = (c >> d) & 1;
                j[d] = i[d] + b;
                if (j[d] == mesh[d]) { j[d] = 0; el.shifts |= 1 << (3 * c + d); }
            }
            cv[c] = ((int64_t)j[2] * n2 + j[1]) * n1 + j[0];
        }
        for (int ca = 0; ca < 8; ++ca) {
            el.bw[ca] = (int32_t)(pl.dof_off[cv[ca] + 1] - pl.dof_off[cv[ca]]);
            for (int cb = 0; cb < 8; ++cb) el.blk[ca * 8 + cb] = block_of(cv[ca], cv[cb]);
        }
        // (atom, descriptor) groups present on the corners
        std::map<std::pair<int, int>, int> gidx;
        for (int c = 0; c < 8; ++c)
            for (int64_t t = pl.vf_off[cv[c]]; t < pl.vf_off[cv[c] + 1]; ++t) gidx[{pl.vf[3 * t], pl.vf[3 * t + 1]}] = 0;
        el.grp_off = (int32_t)pl.groups.size();
        el.ngrp = (int32_t)gidx.size();
        int nfun = 0;
        double centre[3];
        for (int c = 0; c < 3; ++c) centre[c] = (i[0] + 0.5) * E[c] + (i[1] + 0.5) * E[3 + c] + (i[2] + 0.5) * E[6 + c];
        for (auto &kv : gidx) {
            int A = kv.first.first, k = kv.first.second;
            const pufe_enrichment &en = pr.enr[k];
            kv.second = nfun;
            GroupDev g{};
            g.atom = A;
            g.desc = k;
            g.l = en.l;
            g.fbase = nfun;
            g.a = en.a;
            g.rc = en.rc;
            if (en.radial_kind == 1) {
                g.nspl = (int32_t)pr.radial[k].size() - 1;
                g.spl_off = pl.spl_off[k];
                g.a = g.nspl / en.rc;
            }
            g.img_off = (int32_t)(pl.img.size() / 3);
            // images whose cutoff sphere can reach the element
            const double *tau = &pr.pos[3 * A];
            double ur[3], uc[3];
            for (int d = 0; d < 3; ++d) {
                ur[d] = tau[0] * pl.inv[d] + tau[1] * pl.inv[3 + d] + tau[2] * pl.inv[6 + d];
                uc[d] = centre[0] * pl.inv[d] + centre[1] * pl.inv[3 + d] + centre[2] * pl.inv[6 + d];
            }
            double reach = en.rc + Re + kImageMargin;
            int lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
                double rad = reach * std::sqrt(pl.inv[d] * pl.inv[d] + pl.inv[3 + d] * pl.inv[3 + d] + pl.inv[6 + d] * pl.inv[6 + d]);
                lo[d] = (int)std::floor(uc[d] - ur[d] - rad) - 1;
                hi[d] = (int)std::ceil(uc[d] - ur[d] + rad) + 1;
            }
            int nimg = 0;
            for (int m3 = lo[2]; m3 <= hi[2]; ++m3)
                for (int m2 = lo[1]; m2 <= hi[1]; ++m2)
                    for (int m1 = lo[0]; m1 <= hi[0]; ++m1) {
                        double C[3];
                        for (int c = 0; c < 3; ++c) C[c] = tau[c] + m1 * lat[c] + m2 * lat[3 + c] + m3 * lat[6 + c];
                        double dx = C[0] - centre[0], dy = C[1] - centre[1], dz = C[2] - centre[2];
                        if (std::sqrt(dx * dx + dy * dy + dz * dz) >= reach) continue;
                        pl.img.push_back(C[0]);
                        pl.img.push_back(C[1]);
                        pl.img.push_back(C[2]);
                        const int32_t nk[4] = {m1, m2, m3, 0};
                        pl.img_nk.insert(pl.img_nk.end(), nk, nk + 4);
                        ++nimg;
                    }
            g.nimg = nimg;
            pl.groups.push_back(g);
            nfun += 2 * en.l + 1;
        }
        const int nfun_re = nfun;   // functions of the (real-part) groups
        if (pl.bloch) {
            // imaginary parts: a copy of every group, its images weighted by
            // sin(2 pi kappa.n) instead of cos, functions nfun .. 2 nfun - 1
            for (int g = 0; g < el.ngrp; ++g) {
                GroupDev c = pl.groups[el.grp_off + g];
                const int src = c.img_off;
                c.img_off = (int32_t)(pl.img.size() / 3);
                c.fbase += nfun_re;
                for (int k = 0; k < c.nimg; ++k) {
                    for (int t = 0; t < 3; ++t) pl.img.push_back(pl.img[3 * (src + k) + t]);
                    const int32_t nk[4] = {pl.img_nk[4 * (src + k)], pl.img_nk[4 * (src + k) + 1],
                                           pl.img_nk[4 * (src + k) + 2], 1};
                    pl.img_nk.insert(pl.img_nk.end(), nk, nk + 4);
                }
                pl.groups.push_back(c);
            }
            el.ngrp *= 2;
            nfun *= 2;
        }
        el.nfun = nfun;
        if (el.ngrp > 0) pl.max_img = std::max(pl.max_img, (int)(pl.img.size() / 3) - pl.groups[el.grp_off].img_off);
        // enriched local functions: corner by corner, vertex order (with the
        // Bloch-periodic enrichment, a corner's real parts, then its
        // imaginary parts in the same order)
        el.edof_off = (int32_t)pl.edof.size();
        int nenr = 0;
        for (int c = 0; c < 8; ++c) {
            const int64_t t0 = pl.vf_off[cv[c]], t1 = pl.vf_off[cv[c] + 1];
            const int parts = pl.bloch ? 2 : 1;
            for (int part = 0; part < parts; ++part)
                for (int64_t t = t0; t < t1; ++t) {
                    int f = gidx[{pl.vf[3 * t], pl.vf[3 * t + 1]}] + (pl.vf[3 * t + 2] + pr.enr[pl.vf[3 * t + 1]].l);
                    int slot = pl.nfs + (int)(t - t0);
                    pl.edof.push_back(edof_pack(c, f + part * nfun_re, slot));
                    if (pl.bloch) pl.bpart.push_back(part == 0 ? nenr + (int32_t)(t1 - t0) : -1);
                    ++nenr;
                }
        }
        el.nfe = pl.nfe;
        el.nloc = pl.nfe + nenr;
        if (el.nloc > kMaxNloc || nfun > kMaxFun || el.ngrp > kMaxGroups) {
            err = "element " + std::to_string(e) + " holds more functions than the kernels support (nloc " +
                  std::to_string(el.nloc) + ", functions " + std::to_string(nfun) +
                  (pl.bloch ? ", counting real and imaginary parts of the Bloch-periodic enrichment)" : ")");
            return PUFE_ERR_UNSUPPORTED;
        }
        // projector-image groups of the element
        el.pg_off = (int32_t)pl.pgroups.size();
        el.npg = (int32_t)elem_pimg[e].size();
        el.ncol = 0;
        el.pf_nchunk = 0;
        el.pf_base = 0;
        for (const PImg &pi : elem_pimg[e]) {
            PGroupDev g{};
            for (int c = 0; c < 3; ++c) g.c[c] = pi.C[c];
            g.a = pr.proj[pi.d].a;
            g.rc = pr.proj[pi.d].rc;
            g.l = pr.proj[pi.d].l;
            g.col0 = el.ncol;
            g.J0 = pfun_of[pi.d][pi.A];
            for (int d = 0; d < 3; ++d) g.n[d] = pi.n[d];
            pl.pgroups.push_back(g);
            el.ncol += 2 * g.l + 1;
        }
        if (el.ncol > kMaxProjCols || el.npg > kMaxPGroups) {
            err = "element " + std::to_string(e) + " is reached by more projector columns than the kernels hold (" +
                  std::to_string(el.ncol) + ")";
            return PUFE_ERR_UNSUPPORTED;
        }
        pl.max_ncol = std::max(pl.max_ncol, el.ncol);
        pl.max_npg = std::max(pl.max_npg, el.npg);
        pl.max_nloc = std::max(pl.max_nloc, el.nloc);
        pl.max_nfun = std::max(pl.max_nfun, nfun);
        pl.max_ngrp = std::max(pl.max_ngrp, el.ngrp);
        // colour: elements of one colour share no vertex, so their scatters
        // touch disjoint blocks (odd n_d puts the last layer in colour 2)
        int col[3];
        for (int d = 0; d < 3; ++d) col[d] = (mesh[d] % 2 == 1 && i[d] == mesh[d] - 1) ? 2 : (i[d] % 2);
        el.color = col[0] + 3 * col[1] + 9 * col[2];
        by_color[el.color].push_back((int32_t)e);
    }
    pl.img_cur = pl.img;
    // (element, local function) pairs of every DOF, element order
    {
        std::vector<std::vector<int2>> lists(pl.dof_off[pl.nv]);
        for (int64_t e = 0; e < pl.nel; ++e) {
            const ElemDev &el = pl.elems[e];
            for (int a = 0; a < el.nloc; ++a) {
                int corner, slot;
                if (a < el.nfe) {
                    if (pr.p == 1 || (pr.p == 3 && a < 8)) {
                        corner = a;
                        slot = 0;
                    } else if (pr.p == 3) {   // edge node: 8 + 2 e + t, edge e = 4 d + k
                        const int e2 = (a - 8) >> 1, d = e2 >> 2;
                        corner = serendipity_edge_corner(d, e2 & 3);
                        slot = 1 + 2 * d + ((a - 8) & 1);
                    } else {
                        const int d0 = a % 3, d1 = (a / 3) % 3, d2 = a / 9;
                        corner = (d0 == 2) | ((d1 == 2) << 1) | ((d2 == 2) << 2);
                        slot = (d0 == 1) | ((d1 == 1) << 1) | ((d2 == 1) << 2);
                    }
                } else {
                    const int32_t pk = pl.edof[el.edof_off + (a - el.nfe)];
                    corner = pk & 7;
                    slot = pk >> 11;
                }
                lists[pl.dof_off[corner_vertex(e, corner)] + slot].push_back(make_int2((int)e, a));
            }
        }
        pl.dof_el_off.assign(lists.size() + 1, 0);
        pl.dof_el.clear();
        for (size_t g = 0; g < lists.size(); ++g) {
            pl.dof_el.insert(pl.dof_el.end(), lists[g].begin(), lists[g].end());
            pl.dof_el_off[g + 1] = (int64_t)pl.dof_el.size();
        }
    }
    // the scatter relies on elements of one colour sharing no vertex
    {
        std::vector<int32_t> owner(pl.nv * 27, -1);
        for (int64_t e = 0; e < pl.nel; ++e) {
            const ElemDev &el = pl.elems[e];
            for (int c = 0; c < 8; ++c) {
                int j[3];
                for (int d = 0; d < 3; ++d) j[d] = (el.ijk[d] + ((c >> d) & 1)) % mesh[d];
                int64_t v = ((int64_t)j[2] * n2 + j[1]) * n1 + j[0];
                int32_t &o = owner[v * 27 + el.color];
                if (o >= 0 && o != (int32_t)e) { err = "internal error: element colouring conflict"; return PUFE_ERR_INVALID_ARG; }
                o = (int32_t)e;
            }
        }
    }
    pl.color_elems.clear();
    pl.color_off.assign(1, 0);
    pl.scat.clear();
    pl.scat_off.assign(1, 0);
    for (int c = 0; c < 27; ++c) {
        if (by_color[c].empty()) continue;
        pl.color_elems.insert(pl.color_elems.end(), by_color[c].begin(), by_color[c].end());
        pl.color_off.push_back((int32_t)pl.color_elems.size());
        for (int32_t e : by_color[c]) {
            const int T = (pl.elems[e].nloc + 15) / 16;
            for (int p = 0; p < T * (T + 1) / 2; ++p) pl.scat.push_back(make_int2(e, p));
        }
        pl.scat_off.push_back((int64_t)pl.scat.size());
    }

    // ---- kernel constants
    KParams &kp = pl.kp;
    std::memset(&kp, 0, sizeof kp);
    std::memcpy(kp.E, E, sizeof E);
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) kp.Jt[3 * c + d] = 2.0 * mesh[d] * pl.inv[3 * c + d];
    kp.jac = pl.vol / (8.0 * n1 * n2 * n3);
    kp.n = q.n_gauss;
    kp.n3 = q.n_gauss * q.n_gauss * q.n_gauss;
    kp.p = pr.p;
    kp.nfe = pl.nfe;
    kp.nfs = pl.nfs;
    for (int d = 0; d < 3; ++d) kp.mesh[d] = mesh[d];
    // Gauss-Legendre nodes (ascending) and weights: Newton iteration on the
    // three-term Legendre recurrence from cosine initial guesses
    auto gauss = [](int n, double *gx, double *gw) {
        for (int r = 0; r < n; ++r) {
            double x = -std::cos(M_PI * (r + 0.75) / (n + 0.5));
            double dp = 1;
            for (int it = 0; it < 65; ++it) {
                double p0 = 1, p1 = x;
                for (int k = 1; k < n; ++k) {
                    double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
                    p0 = p1;
                    p1 = p2;
                }
                if (n == 1) { p0 = 1; p1 = x; }
                dp = n * (p0 - x * p1) / (1 - x * x);
                if (it == 64) break;
                double dx = p1 / dp;
                x -= dx;
                if (std::fabs(dx) < 1e-16) it = 63;   // one more pass refreshes dp at the root
            }
            gx[r] = x;
            gw[r] = 2.0 / ((1 - x * x) * dp * dp);
        }
    };
    gauss(q.n_gauss, kp.gx, kp.gw);
    kp.nref = q.mode == PUFE_QUAD_ERROR ? q.n_ref : 0;
    if (kp.nref > 0) gauss(kp.nref, kp.rx, kp.rw);
    return PUFE_OK;
}

}  // namespace pufe
