// C ABI of the PUFE assembly library (declared in include/pufe.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pufe.h"
#include "aq_error.hpp"
#include "backward.hpp"
#include "bloch.hpp"
#include "kernels.hpp"
#include "nonlocal.hpp"
#include "plan.hpp"
#include "scf.hpp"

using namespace pufe;

namespace {

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t count) {
        release();
        if (count == 0) count = 1;
        hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
        if (e == hipSuccess) n = count;
        else p = nullptr;
        return e;
    }
    hipError_t upload(const std::vector<T> &v, hipStream_t st) {
        hipError_t e = alloc(v.size());
        if (e != hipSuccess || v.empty()) return e;
        e = hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(st);
    }
};

}  // namespace

struct pufe_ctx {
    int device = 0;
    std::string err;
    bool have_problem = false, have_setup = false;
    Problem prob;
    Plan plan;
    int64_t n_leaves = 0, n_qp = 0;
    std::vector<int64_t> leaf_off_h;
    std::vector<ItemDev> items, items_split;
    // wide work items: the row and column blocks of elements of more than
    // kWholeMaxTiles tiles, for the 8-wave kernel (wide_tiles = 0: none, those
    // elements go to the narrow kernel)
    std::vector<ItemDev> items_wide;
    int wide_tiles = kWideTiles, max_rows_wide = 16, max_item_leaves_wide = 1;
    size_t lds_wide = 0;
    size_t lds = 0;
    int max_rows = 16, max_rows_split = 16, max_item_leaves_split = 1;
    int64_t part_slots = 0;
    double tune_items = 4096.0;
    int tune_block = kBlockTiles;
    bool tuned = false;             // item plan and stage length chosen by pufe_tune
    int contract_q = 24;            // points per LDS stage of the FP64 contraction (16, 24 or 32)
    int max_item_leaves = 1;
    // bumped whenever the device tables or work items are rebuilt (problem,
    // setup, tuner): a batch created earlier refuses to run on a newer plan
    uint64_t plan_gen = 0;
    DevBuf<ElemDev> d_elems;
    DevBuf<GroupDev> d_groups;
    DevBuf<double> d_img, d_pos, d_partial;
    DevBuf<double> d_spl;           // coefficients of the tabulated radials
    DevBuf<int32_t> d_edof, d_leaf_elem, d_color_elems, d_brow, d_bcol;
    DevBuf<int2> d_scat;
    std::vector<int2> reduce;       // (element, tile pair) of every element with several K-chunks
    DevBuf<int2> d_reduce;
    DevBuf<double2> d_ztab;
    DevBuf<uint32_t> d_leaves;
    DevBuf<int64_t> d_leaf_count, d_leaf_off, d_bval_off, d_dof_off;
    DevBuf<ItemDev> d_items, d_items_split, d_items_wide;
    // adjoint
    bool have_bw = false;
    std::vector<ItemDev> bw_items, bw_items_wide;   // elements of <= 80 functions, and the rest
    size_t bw_lds = 0, bw_lds_wide = 0;
    DevBuf<ItemDev> d_bw_items, d_bw_items_wide;
    DevBuf<int64_t> d_pt_off, d_atom_ptr, d_atom_slots;
    DevBuf<double> d_Pt, d_fP, d_fQ;
    // separable nonlocal term
    std::vector<NlItemDev> nl_items;
    std::vector<int32_t> nl_elems;
    int64_t nl_doubles = 0;
    size_t nl_lds = 0;
    DevBuf<NlItemDev> d_nl_items;
    DevBuf<PGroupDev> d_pgroups;
    DevBuf<double> d_Fp, d_pfun_h;
    DevBuf<int64_t> d_dof_el_off;
    DevBuf<int2> d_dof_el;
    DevBuf<int32_t> d_nl_elems, d_nl_blocks;
    DevBuf<double2> d_nlf;
    // Bloch-periodic enrichment: image shifts and kinds, the per-k image
    // weights, the partner table of the enriched entries
    DevBuf<int32_t> d_img_nk, d_bpart;
    DevBuf<double> d_wimg;
    // self-consistent field pieces: per-element load sums, the classical FE
    // blocks of the stiffness matrix, the FE integrals m_i, CG workspace
    DevBuf<double> d_fe_be, d_Kfe, d_mfe, d_fe_ones, d_cg, d_dot;
    DevBuf<int64_t> d_brow_ptr;
    bool have_poisson = false;
    double m_sum = 0.0;
    // timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[5];
    ~pufe_ctx() { clear_events(); }
    void clear_events() {
        for (auto &v : ev) {
            for (auto &pr : v) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
            v.clear();
        }
    }
};

// Bracket the launches enqueued between begin() and end() with events when
// timing is on.
struct TimedRegion {
    pufe_ctx *c;
    int slot;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    TimedRegion(pufe_ctx *c_, int s, hipStream_t st_) : c(c_), slot(s), st(st_) {
        if (!c->timing || slot < 0) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
        (void)hipEventRecord(a, st);
    }
    ~TimedRegion() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        c->ev[slot].push_back({a, b});
    }
};

static int fail(pufe_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

static int hipfail(pufe_ctx *c, hipError_t e, const char *where) {
    int code = (e == hipErrorOutOfMemory) ? PUFE_ERR_OOM : PUFE_ERR_HIP;
    return fail(c, code, std::string(where) + ": " + hipGetErrorString(e));
}

#define CHECK_HIP(ctx, x, where)                          \
    do {                                                  \
        hipError_t e_ = (x);                              \
        if (e_ != hipSuccess) return hipfail(ctx, e_, where); \
    } while (0)

extern "C" {

const char *pufe_error_string(int code) {
    switch (code) {
        case PUFE_OK: return "ok";
        case PUFE_ERR_INVALID_ARG: return "invalid argument";
        case PUFE_ERR_UNSUPPORTED: return "unsupported";
        case PUFE_ERR_OOM: return "out of device memory";
        case PUFE_ERR_HIP: return "HIP runtime error";
        case PUFE_ERR_STATE: return "call out of order";
        default: return "unknown error";
    }
}

const char *pufe_last_error_message(const pufe_ctx *ctx) {
    if (!ctx) return "no context";
    return ctx->err.c_str();
}

int pufe_create(pufe_ctx **out, int device) {
    if (!out) return PUFE_ERR_INVALID_ARG;
    if (device < 0) return PUFE_ERR_INVALID_ARG;
    pufe_ctx *c = new (std::nothrow) pufe_ctx();
    if (!c) return PUFE_ERR_OOM;
    c->device = device;
    *out = c;
    return PUFE_OK;
}

int pufe_destroy(pufe_ctx *ctx) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (ctx->have_setup) (void)hipSetDevice(ctx->device);
    delete ctx;
    return PUFE_OK;
}

int pufe_set_problem(pufe_ctx *ctx, const double lattice[9], const int mesh[3], int fe_order, int n_atoms,
                     const double *pos, const int *species, int n_enr, const pufe_enrichment *enr,
                     const pufe_quad *quad) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!lattice || !mesh || !quad || n_atoms < 0 || n_enr < 0 || (n_atoms > 0 && (!pos || !species)) ||
        (n_enr > 0 && !enr))
        return fail(ctx, PUFE_ERR_INVALID_ARG, "null pointer or negative count");
    Problem pr;
    std::memcpy(pr.lat, lattice, sizeof pr.lat);
    std::memcpy(pr.mesh, mesh, sizeof pr.mesh);
    pr.p = fe_order;
    pr.pos.assign(pos, pos + 3 * (size_t)n_atoms);
    pr.species.assign(species, species + n_atoms);
    pr.enr.assign(enr, enr + n_enr);
    pr.radial.assign(n_enr, {});
    for (int k = 0; k < n_enr; ++k) {   // keep a copy of the samples, never the caller's pointer
        if (enr[k].radial_kind == 1) {
            if (!enr[k].radial || enr[k].n_radial < 0 || enr[k].n_radial > 4096)
                return fail(ctx, PUFE_ERR_INVALID_ARG, "a tabulated radial needs 4..4096 samples");
            pr.radial[k].assign(enr[k].radial, enr[k].radial + enr[k].n_radial);
        }
        pr.enr[k].radial = nullptr;
        pr.enr[k].n_radial = (int)pr.radial[k].size();
    }
    pr.quad = *quad;
    for (double v : pr.pos)
        if (!std::isfinite(v)) return fail(ctx, PUFE_ERR_INVALID_ARG, "non-finite atom position");
    Plan pl;
    std::string err;
    int rc = build_plan(pr, pl, err);
    if (rc != PUFE_OK) return fail(ctx, rc, err);
    ctx->prob = std::move(pr);
    ctx->plan = std::move(pl);
    ctx->have_problem = true;
    ctx->have_setup = false;
    ctx->have_bw = false;
    ctx->n_leaves = ctx->n_qp = 0;
    ++ctx->plan_gen;
    return PUFE_OK;
}

int pufe_set_projectors(pufe_ctx *ctx, int n, const pufe_projector *proj) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_problem) return fail(ctx, PUFE_ERR_STATE, "pufe_set_problem must come first");
    if (ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "projectors are set before pufe_setup");
    if (n < 0 || (n > 0 && !proj)) return fail(ctx, PUFE_ERR_INVALID_ARG, "null pointer or negative count");
    Problem pr = ctx->prob;
    pr.proj.assign(proj, proj + n);
    Plan pl;
    std::string err;
    int rc = build_plan(pr, pl, err);
    if (rc != PUFE_OK) return fail(ctx, rc, err);
    ctx->prob = std::move(pr);
    ctx->plan = std::move(pl);
    ++ctx->plan_gen;
    return PUFE_OK;
}

int pufe_set_enrichment_phase(pufe_ctx *ctx, int form) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_problem) return fail(ctx, PUFE_ERR_STATE, "pufe_set_problem must come first");
    if (ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "the enrichment form is set before pufe_setup");
    if (form != PUFE_ENR_PERIODIC && form != PUFE_ENR_BLOCH)
        return fail(ctx, PUFE_ERR_INVALID_ARG, "unknown enrichment form");
    Problem pr = ctx->prob;
    pr.enr_phase = form;
    Plan pl;
    std::string err;
    int rc = build_plan(pr, pl, err);
    if (rc != PUFE_OK) return fail(ctx, rc, err);
    ctx->prob = std::move(pr);
    ctx->plan = std::move(pl);
    ++ctx->plan_gen;
    return PUFE_OK;
}

// Split each element's contraction into K-chunks (ranges of leaves) of about
// equal MFMA work; the chunking fixes the layout of the partial tiles and does
// not depend on how the tile pairs of a chunk are grouped into work items.
static void plan_chunks(pufe_ctx *c, double target_items) {
    Plan &pl = c->plan;
    const int n3 = pl.kp.n3;
    double total = 0;
    for (const ElemDev &el : pl.elems) {
        const int T = (el.nloc + 15) / 16;
        total += (double)T * (T + 1) / 2 * n3 * (el.leaf_end - el.leaf_off);
    }
    const double target = std::max(total / target_items, 1.0);
    int64_t base = 0;
    for (ElemDev &el : pl.elems) {
        const int T = (el.nloc + 15) / 16;
        const int64_t P = (int64_t)T * (T + 1) / 2, nleaf = el.leaf_end - el.leaf_off;
        int64_t nch = (int64_t)std::llround((double)nleaf * n3 * P / target);
        nch = std::max<int64_t>(1, std::min<int64_t>(nch, nleaf));
        el.nchunk = (int32_t)nch;
        el.part_base = base;
        base += nch * P;
    }
    c->part_slots = base;
    c->reduce.clear();
    for (int64_t e = 0; e < pl.nel; ++e) {
        const ElemDev &el = pl.elems[e];
        const int T = (el.nloc + 15) / 16;
        if (el.nchunk > 1)
            for (int p = 0; p < T * (T + 1) / 2; ++p) c->reduce.push_back(make_int2((int)e, p));
    }
}

// Work items (row block x column block of 16x16 tiles x K-chunk), largest
// MFMA work first.  sel: 0 every element, 1 the elements of at most
// kWholeMaxTiles tiles, 2 the others.
static std::vector<ItemDev> make_items(const pufe_ctx *c, int block_tiles, int *max_rows, int *max_leaves,
                                       int sel = 0) {
    const Plan &pl = c->plan;
    std::vector<ItemDev> items;
    std::vector<double> cost;
    for (int64_t e = 0; e < pl.nel; ++e) {
        const ElemDev &el = pl.elems[e];
        const int T = (el.nloc + 15) / 16;
        if ((sel == 1 && T > kWholeMaxTiles) || (sel == 2 && T <= kWholeMaxTiles)) continue;
        // up to 5 tiles fit one diagonal block (15 tile pairs over 4 waves)
        const int bt = (T <= 5 && block_tiles >= 4) ? T : block_tiles;
        const int nb = (T + bt - 1) / bt;
        const int64_t nleaf = el.leaf_end - el.leaf_off, nch = el.nchunk;
        for (int64_t ch = 0; ch < nch; ++ch) {
            const int64_t lb = el.leaf_off + ch * nleaf / nch, le = el.leaf_off + (ch + 1) * nleaf / nch;
            for (int bj = 0; bj < nb; ++bj)
                for (int bi = 0; bi <= bj; ++bi) {
                    ItemDev it{};
                    it.elem = (int32_t)e;
                    it.I0 = bi * bt;
                    it.nI = std::min(bt, T - it.I0);
                    it.J0 = bj * bt;
                    it.nJ = std::min(bt, T - it.J0);
                    it.chunk = (int32_t)ch;
                    it.leaf_b = lb;
                    it.leaf_e = le;
                    const int pairs = bi == bj ? it.nI * (it.nI + 1) / 2 : it.nI * it.nJ;
                    items.push_back(it);
                    cost.push_back((double)pairs * (le - lb));
                }
        }
    }
    std::vector<size_t> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    std::vector<ItemDev> sorted;
    sorted.reserve(order.size());
    int rows = 16, leaves = 1;
    for (size_t i : order) {
        sorted.push_back(items[i]);
        rows = std::max(rows, 16 * (items[i].I0 == items[i].J0 ? items[i].nI : items[i].nI + items[i].nJ));
        leaves = std::max(leaves, (int)(items[i].leaf_e - items[i].leaf_b));
    }
    *max_rows = rows;
    if (max_leaves) *max_leaves = leaves;
    return sorted;
}

static void plan_items(pufe_ctx *c, double target_items, int block_tiles) {
    plan_chunks(c, target_items);
    const int nfun = std::max(c->plan.max_nfun, 1);
    const int n3 = c->plan.kp.n3;
    // wide items first: tile blocks of wide_tiles (fewer if the stage does
    // not fit in LDS); without them every element goes to the narrow kernel
    c->items_wide.clear();
    bool wide = false;
    for (int b = c->wide_tiles; b >= 2; --b) {
        c->items_wide = make_items(c, b, &c->max_rows_wide, &c->max_item_leaves_wide, 2);
        c->lds_wide = contract_wide_lds_bytes(c->max_rows_wide, nfun, c->plan.max_img, c->max_item_leaves_wide, n3);
        if (c->lds_wide <= kMaxDynLds) {
            wide = true;
            break;
        }
    }
    if (!wide) c->items_wide.clear();
    // the FP64 stage double-buffers the rows of an item: use the largest
    // tile block (and stage length) whose buffers fit in LDS
    for (int b = block_tiles; b >= 1; --b) {
        c->items = make_items(c, b, &c->max_rows, &c->max_item_leaves, wide ? 1 : 0);
        c->lds = contract_lds_bytes(c->contract_q, c->max_rows, nfun, c->plan.max_img, c->max_item_leaves, n3);
        if (c->lds > kMaxDynLds && c->contract_q > 16) {   // shorter stages before smaller blocks
            c->contract_q = 16;
            c->lds = contract_lds_bytes(16, c->max_rows, nfun, c->plan.max_img, c->max_item_leaves, n3);
        }
        if (c->lds <= kMaxDynLds) break;
    }
    // the split stage keeps bf16 limbs of every row: use the largest tile
    // block whose three-limb stage fits in LDS
    for (int b = block_tiles; b >= 1; --b) {
        c->items_split = make_items(c, b, &c->max_rows_split, &c->max_item_leaves_split);
        if (split_lds_bytes(3, c->max_rows_split, nfun, c->plan.max_img, c->max_item_leaves_split, n3) <= kMaxDynLds)
            break;
    }
    // nonlocal work items: the contraction's K-chunks of every element a
    // projector image reaches, cut into row blocks of at most 16 tile pairs
    // (row tiles x projector column tiles); one coefficient slot per chunk
    c->nl_items.clear();
    c->nl_elems.clear();
    c->nl_doubles = 0;
    int max_npad = 16, max_leaves = 1;
    for (int64_t e = 0; e < c->plan.nel; ++e) {
        ElemDev &el = c->plan.elems[e];
        el.pf_nchunk = 0;
        el.pf_base = 0;
        if (el.npg == 0) continue;
        const int T = (el.nloc + 15) / 16, TC = (el.ncol + 15) / 16, RB = std::max(1, 16 / TC);
        const int64_t nleaf = el.leaf_end - el.leaf_off, nch = el.nchunk;
        el.pf_nchunk = (int32_t)nch;
        el.pf_base = c->nl_doubles;
        c->nl_doubles += nch * (int64_t)(16 * TC) * (16 * T);
        c->nl_elems.push_back((int32_t)e);
        max_npad = std::max(max_npad, 16 * T);
        for (int64_t ch = 0; ch < nch; ++ch)
            for (int R0 = 0; R0 < T; R0 += RB) {
                NlItemDev it{};
                it.elem = (int32_t)e;
                it.chunk = (int32_t)ch;
                it.R0 = R0;
                it.nR = std::min(RB, T - R0);
                it.leaf_b = el.leaf_off + ch * nleaf / nch;
                it.leaf_e = el.leaf_off + (ch + 1) * nleaf / nch;
                max_leaves = std::max(max_leaves, (int)(it.leaf_e - it.leaf_b));
                c->nl_items.push_back(it);
            }
    }
    c->nl_lds = nl_lds_bytes(max_npad, std::max(c->plan.max_ncol, 1), nfun, c->plan.max_img, max_leaves, n3);
}

static int upload_items(pufe_ctx *ctx, hipStream_t st);

// Device tables and buffers of the nonlocal term for the current plan.
static int upload_nonlocal(pufe_ctx *ctx, hipStream_t st) {
    const Plan &pl = ctx->plan;
    if (pl.n_pfun == 0) return PUFE_OK;
    if (ctx->nl_lds > kMaxDynLds) return fail(ctx, PUFE_ERR_UNSUPPORTED, "nonlocal stage does not fit in LDS");
    CHECK_HIP(ctx, ctx->d_nl_items.upload(ctx->nl_items, st), "upload nonlocal items");
    CHECK_HIP(ctx, ctx->d_nl_elems.upload(ctx->nl_elems, st), "upload nonlocal elements");
    CHECK_HIP(ctx, ctx->d_pgroups.upload(pl.pgroups, st), "upload projector groups");
    CHECK_HIP(ctx, ctx->d_pfun_h.upload(pl.pfun_h, st), "upload projector weights");
    CHECK_HIP(ctx, ctx->d_dof_el_off.upload(pl.dof_el_off, st), "upload DOF map");
    CHECK_HIP(ctx, ctx->d_dof_el.upload(pl.dof_el, st), "upload DOF map");
    CHECK_HIP(ctx, ctx->d_nl_blocks.upload(pl.nl_blocks, st), "upload nonlocal blocks");
    CHECK_HIP(ctx, ctx->d_Fp.alloc((size_t)std::max<int64_t>(ctx->nl_doubles, 1)), "alloc projector coefficients");
    CHECK_HIP(ctx, ctx->d_nlf.alloc((size_t)kMaxKPerLaunch * pl.n_pfun * pl.dof_off[pl.nv]), "alloc projector sums");
    return PUFE_OK;
}

int pufe_setup(pufe_ctx *ctx, void *stream) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_problem) return fail(ctx, PUFE_ERR_STATE, "pufe_set_problem must come first");
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    {
        hipError_t ea = init_contract_attributes();
        if (ea == hipSuccess) ea = init_split_attributes();
        if (ea == hipSuccess) ea = init_backward_attributes();
        if (ea == hipSuccess) ea = init_nonlocal_attributes();
        if (ea != hipSuccess) {
            (void)hipGetLastError();   // do not leave the error for the caller's next HIP call
            return hipfail(ctx, ea, "kernel attributes");
        }
    }
    Plan &pl = ctx->plan;
    const int64_t nel = pl.nel;
    const int n_atoms = (int)ctx->prob.species.size();
    CHECK_HIP(ctx, ctx->d_pos.upload(ctx->prob.pos, st), "upload positions");
    CHECK_HIP(ctx, ctx->d_spl.upload(pl.spl, st), "upload radial tables");
    pl.kp.spl = ctx->d_spl.p;
    CHECK_HIP(ctx, ctx->d_leaf_count.alloc(nel + 1), "alloc leaf counts");
    CHECK_HIP(ctx, ctx->d_leaf_off.alloc(nel + 1), "alloc leaf offsets");
    const double L[3] = {pl.lat[0], pl.lat[4], pl.lat[8]};
    const pufe_quad &q = ctx->prob.quad;
    ctx->leaf_off_h.assign(nel + 1, 0);
    if (q.mode == PUFE_QUAD_GEOM) {
        // count leaves, scan, emit (one octree walk per element, twice)
        CHECK_HIP(ctx, launch_aq_geom(pl.kp, nel, ctx->d_pos.p, n_atoms, L, q.max_level, q.dist, ctx->d_leaf_count.p,
                                      nullptr, nullptr, nullptr, st), "adaptive quadrature (count)");
        CHECK_HIP(ctx, launch_scan(ctx->d_leaf_count.p, nel, ctx->d_leaf_off.p, st), "scan");
        CHECK_HIP(ctx, hipMemcpyAsync(ctx->leaf_off_h.data(), ctx->d_leaf_off.p, sizeof(int64_t) * (nel + 1),
                                      hipMemcpyDeviceToHost, st), "download leaf offsets");
        CHECK_HIP(ctx, hipStreamSynchronize(st), "sync");
        ctx->n_leaves = ctx->leaf_off_h[nel];
        CHECK_HIP(ctx, ctx->d_leaves.alloc(ctx->n_leaves), "alloc leaves");
        CHECK_HIP(ctx, ctx->d_leaf_elem.alloc(ctx->n_leaves), "alloc leaf elements");
        CHECK_HIP(ctx, launch_aq_geom(pl.kp, nel, ctx->d_pos.p, n_atoms, L, q.max_level, q.dist, nullptr,
                                      ctx->d_leaf_off.p, ctx->d_leaves.p, ctx->d_leaf_elem.p, st),
                  "adaptive quadrature (emit)");
    } else {
        // error-driven rule: the element tables are needed first
        DevBuf<ElemDev> elems;
        CHECK_HIP(ctx, elems.upload(pl.elems, st), "upload elements");
        CHECK_HIP(ctx, ctx->d_groups.upload(pl.groups, st), "upload groups");
        CHECK_HIP(ctx, ctx->d_img.upload(pl.img_cur, st), "upload images");
        DevBuf<CellDev> cur, next;
        DevBuf<int64_t> cnt, off;
        DevBuf<uint64_t> nmask;
        CHECK_HIP(ctx, cur.alloc(nel), "alloc cells");
        CHECK_HIP(ctx, launch_aq_error_init(nel, elems.p, cur.p, st), "rule roots");
        int64_t n = nel;
        for (int lev = 0; lev < q.max_level; ++lev) {
            CHECK_HIP(ctx, cnt.alloc(n + 1), "alloc counts");
            CHECK_HIP(ctx, off.alloc(n + 1), "alloc offsets");
            CHECK_HIP(ctx, nmask.alloc(n + 1), "alloc masks");
            CHECK_HIP(ctx, launch_aq_error_test(pl.kp, elems.p, ctx->d_groups.p, ctx->d_img.p, cur.p, n, q.max_level,
                                                q.tol, cnt.p, nmask.p, st), "rule test");
            CHECK_HIP(ctx, launch_scan(cnt.p, n, off.p, st), "scan");
            int64_t total = 0;
            CHECK_HIP(ctx, hipMemcpyAsync(&total, off.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, st), "download");
            CHECK_HIP(ctx, hipStreamSynchronize(st), "sync");
            if (total == n) break;   // no cell split at this level
            CHECK_HIP(ctx, next.alloc(total), "alloc cells");
            CHECK_HIP(ctx, launch_aq_error_expand(n, cur.p, off.p, nmask.p, next.p, st), "rule expand");
            std::swap(cur.p, next.p);
            std::swap(cur.n, next.n);
            n = total;
        }
        ctx->n_leaves = n;
        CHECK_HIP(ctx, ctx->d_leaves.alloc(n), "alloc leaves");
        CHECK_HIP(ctx, ctx->d_leaf_elem.alloc(n), "alloc leaf elements");
        CHECK_HIP(ctx, launch_aq_error_finish(n, cur.p, ctx->d_leaves.p, ctx->d_leaf_elem.p, ctx->d_leaf_count.p, st),
                  "rule leaves");
        CHECK_HIP(ctx, launch_scan(ctx->d_leaf_count.p, nel, ctx->d_leaf_off.p, st), "scan");
        CHECK_HIP(ctx, hipMemcpyAsync(ctx->leaf_off_h.data(), ctx->d_leaf_off.p, sizeof(int64_t) * (nel + 1),
                                      hipMemcpyDeviceToHost, st), "download leaf offsets");
        CHECK_HIP(ctx, hipStreamSynchronize(st), "sync");
    }
    ctx->n_qp = ctx->n_leaves * pl.kp.n3;
    for (int64_t e = 0; e < nel; ++e) {
        pl.elems[e].leaf_off = ctx->leaf_off_h[e];
        pl.elems[e].leaf_end = ctx->leaf_off_h[e + 1];
    }
    plan_items(ctx, ctx->tune_items, ctx->tune_block);
    if (ctx->lds > kMaxDynLds)
        return fail(ctx, PUFE_ERR_UNSUPPORTED, "contraction stage does not fit in LDS");
    CHECK_HIP(ctx, ctx->d_elems.upload(pl.elems, st), "upload elements");
    CHECK_HIP(ctx, ctx->d_groups.upload(pl.groups, st), "upload groups");
    CHECK_HIP(ctx, ctx->d_img.upload(pl.img_cur, st), "upload images");
    CHECK_HIP(ctx, ctx->d_edof.upload(pl.edof, st), "upload enriched functions");
    CHECK_HIP(ctx, ctx->d_img_nk.upload(pl.img_nk, st), "upload image shifts");
    CHECK_HIP(ctx, ctx->d_bpart.upload(pl.bpart, st), "upload enriched partners");
    CHECK_HIP(ctx, ctx->d_wimg.alloc(pl.bloch ? pl.img_nk.size() / 4 : 0), "alloc image weights");
    CHECK_HIP(ctx, ctx->d_items.upload(ctx->items, st), "upload work items");
    CHECK_HIP(ctx, ctx->d_items_wide.upload(ctx->items_wide, st), "upload work items");
    CHECK_HIP(ctx, ctx->d_items_split.upload(ctx->items_split, st), "upload work items");
    // tables of the self-consistent field pieces belong to the previous plan
    ctx->d_dof_el_off.release();
    ctx->d_dof_el.release();
    ctx->d_fe_be.release();
    ctx->have_poisson = false;
    {
        int rc = upload_nonlocal(ctx, st);
        if (rc != PUFE_OK) return rc;
    }
    CHECK_HIP(ctx, ctx->d_color_elems.upload(pl.color_elems, st), "upload colours");
    CHECK_HIP(ctx, ctx->d_scat.upload(pl.scat, st), "upload scatter list");
    CHECK_HIP(ctx, ctx->d_reduce.upload(ctx->reduce, st), "upload chunk reduction list");
    CHECK_HIP(ctx, ctx->d_ztab.alloc(kMaxKPerLaunch * 27), "alloc phase table");
    CHECK_HIP(ctx, ctx->d_brow.upload(pl.brow, st), "upload layout");
    CHECK_HIP(ctx, ctx->d_bcol.upload(pl.bcol, st), "upload layout");
    CHECK_HIP(ctx, ctx->d_bval_off.upload(pl.bval_off, st), "upload layout");
    CHECK_HIP(ctx, ctx->d_dof_off.upload(pl.dof_off, st), "upload layout");
    CHECK_HIP(ctx, ctx->d_partial.alloc((size_t)ctx->part_slots * 512), "alloc partial tiles");
    {
        // the allocation-free entry's workspace: its device address is looked
        // up once per device, here at set-up
        double *ws = nullptr;
        CHECK_HIP(ctx, scratch_address(ctx->device, &ws), "workspace address");
    }
    CHECK_HIP(ctx, hipStreamSynchronize(st), "sync");
    ctx->have_setup = true;
    ++ctx->plan_gen;
    return PUFE_OK;
}

int pufe_set_rule(pufe_ctx *ctx, int64_t n_leaves, const int32_t *level, const int32_t *ijk,
                  const int64_t *elem_leaf_offset, void *stream) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "pufe_setup must come first");
    Plan &pl = ctx->plan;
    const int64_t nel = pl.nel;
    if (n_leaves < nel || !level || !ijk || !elem_leaf_offset)
        return fail(ctx, PUFE_ERR_INVALID_ARG, "null pointer or fewer leaves than elements");
    if (elem_leaf_offset[0] != 0 || elem_leaf_offset[nel] != n_leaves)
        return fail(ctx, PUFE_ERR_INVALID_ARG, "leaf offsets must run from 0 to n_leaves");
    std::vector<uint32_t> codes(n_leaves);
    std::vector<int32_t> lelem(n_leaves);
    for (int64_t e = 0; e < nel; ++e) {
        const int64_t b = elem_leaf_offset[e], en = elem_leaf_offset[e + 1];
        if (en <= b) return fail(ctx, PUFE_ERR_INVALID_ARG, "every element needs at least one leaf");
        // the leaves of an element tile its reference cube: their volumes,
        // in units of the finest cell, add up to the whole
        int64_t vol = 0;
        for (int64_t k = b; k < en; ++k) {
            const int lev = level[k];
            if (lev < 0 || lev > kMaxLevel) return fail(ctx, PUFE_ERR_INVALID_ARG, "leaf level outside 0..8");
            for (int d = 0; d < 3; ++d)
                if (ijk[3 * k + d] < 0 || ijk[3 * k + d] >= (1 << lev))
                    return fail(ctx, PUFE_ERR_INVALID_ARG, "leaf coordinate outside its level's range");
            vol += (int64_t)1 << (3 * (kMaxLevel - lev));
            codes[k] = leaf_pack(lev, ijk[3 * k], ijk[3 * k + 1], ijk[3 * k + 2]);
            lelem[k] = (int32_t)e;
        }
        if (vol != (int64_t)1 << (3 * kMaxLevel))
            return fail(ctx, PUFE_ERR_INVALID_ARG, "the leaves of an element do not cover its cell once");
    }
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    CHECK_HIP(ctx, hipStreamSynchronize(st), "sync");
    CHECK_HIP(ctx, ctx->d_leaves.alloc(n_leaves), "alloc leaves");
    CHECK_HIP(ctx, ctx->d_leaf_elem.alloc(n_leaves), "alloc leaf elements");
    CHECK_HIP(ctx, hipMemcpy(ctx->d_leaves.p, codes.data(), sizeof(uint32_t) * n_leaves, hipMemcpyHostToDevice),
              "upload leaves");
    CHECK_HIP(ctx, hipMemcpy(ctx->d_leaf_elem.p, lelem.data(), sizeof(int32_t) * n_leaves, hipMemcpyHostToDevice),
              "upload leaf elements");
    ctx->leaf_off_h.assign(elem_leaf_offset, elem_leaf_offset + nel + 1);
    CHECK_HIP(ctx, hipMemcpy(ctx->d_leaf_off.p, ctx->leaf_off_h.data(), sizeof(int64_t) * (nel + 1),
                             hipMemcpyHostToDevice), "upload leaf offsets");
    ctx->n_leaves = n_leaves;
    ctx->n_qp = n_leaves * pl.kp.n3;
    for (int64_t e = 0; e < nel; ++e) {
        pl.elems[e].leaf_off = ctx->leaf_off_h[e];
        pl.elems[e].leaf_end = ctx->leaf_off_h[e + 1];
    }
    plan_items(ctx, ctx->tune_items, ctx->tune_block);
    if (ctx->lds > kMaxDynLds) return fail(ctx, PUFE_ERR_UNSUPPORTED, "contraction stage does not fit in LDS");
    return upload_items(ctx, nullptr);
}

int pufe_query(pufe_ctx *ctx, pufe_sizes *out) {
    if (!ctx || !out) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_problem) return fail(ctx, PUFE_ERR_STATE, "no problem defined");
    const Plan &pl = ctx->plan;
    std::memset(out, 0, sizeof *out);
    out->n_elem = pl.nel;
    out->n_vertex = pl.nv;
    out->n_dof = pl.dof_off[pl.nv];
    out->n_fe_dof = pl.nv * pl.nfs;
    out->n_enr_dof = out->n_dof - out->n_fe_dof;
    out->nnzb = (int64_t)pl.bcol.size();
    out->nnz = pl.nnz;
    out->n_qp = ctx->n_qp;
    out->n_leaves = ctx->n_leaves;
    out->max_nloc = pl.max_nloc;
    out->n_colors = (int32_t)pl.color_off.size() - 1;
    out->n_atoms = (int32_t)ctx->prob.species.size();
    out->n_fe_slots = pl.nfs;
    return PUFE_OK;
}

int pufe_get_layout(pufe_ctx *ctx, int64_t *dof_offset, int64_t *brow_ptr, int32_t *bcol, int64_t *bval_offset) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_problem) return fail(ctx, PUFE_ERR_STATE, "no problem defined");
    const Plan &pl = ctx->plan;
    if (dof_offset) std::memcpy(dof_offset, pl.dof_off.data(), sizeof(int64_t) * pl.dof_off.size());
    if (brow_ptr) std::memcpy(brow_ptr, pl.brow_ptr.data(), sizeof(int64_t) * pl.brow_ptr.size());
    if (bcol) std::memcpy(bcol, pl.bcol.data(), sizeof(int32_t) * pl.bcol.size());
    if (bval_offset) std::memcpy(bval_offset, pl.bval_off.data(), sizeof(int64_t) * pl.bval_off.size());
    return PUFE_OK;
}

int pufe_get_quadrature(pufe_ctx *ctx, double *d_xyz, double *d_w, int64_t *d_elem_qp_offset, void *stream) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "pufe_setup must come first");
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (d_xyz || d_w)
        CHECK_HIP(ctx, launch_qp_export(ctx->plan.kp, ctx->n_leaves, ctx->d_leaves.p, ctx->d_leaf_elem.p, d_xyz, d_w, st),
                  "quadrature export");
    if (d_elem_qp_offset)
        CHECK_HIP(ctx, launch_elem_qp_offset(ctx->plan.kp, ctx->plan.nel, ctx->d_leaf_off.p, d_elem_qp_offset, st),
                  "quadrature offsets");
    return PUFE_OK;
}

int pufe_get_leaves(pufe_ctx *ctx, int32_t *level, int32_t *ijk, int64_t *elem_leaf_offset) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "pufe_setup must come first");
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    std::vector<uint32_t> codes(std::max<int64_t>(ctx->n_leaves, 1));
    CHECK_HIP(ctx, hipMemcpy(codes.data(), ctx->d_leaves.p, sizeof(uint32_t) * ctx->n_leaves, hipMemcpyDeviceToHost),
              "download leaves");
    for (int64_t i = 0; i < ctx->n_leaves; ++i) {
        uint32_t c = codes[i];
        if (level) level[i] = (int32_t)(c >> 27);
        if (ijk) {
            ijk[3 * i] = (int32_t)(c & 511u);
            ijk[3 * i + 1] = (int32_t)((c >> 9) & 511u);
            ijk[3 * i + 2] = (int32_t)((c >> 18) & 511u);
        }
    }
    if (elem_leaf_offset) std::memcpy(elem_leaf_offset, ctx->leaf_off_h.data(), sizeof(int64_t) * ctx->leaf_off_h.size());
    return PUFE_OK;
}

// Problems with tabulated radials, serendipity elements or the Bloch-periodic
// enrichment run the general variant of the contraction kernels; the others a
// variant compiled for analytic radials and Lagrange elements only (fewer
// live registers).
static bool general_variant(const Plan &pl) { return !pl.spl.empty() || pl.kp.p == 3 || pl.bloch; }

// The element contraction and the K-chunk sum into `partial` (the context's
// partial-tile buffer, or the fixed workspace of the allocation-free entry);
// wimg: image weights of the Bloch-periodic enrichment at one k-point (null
// for the periodic form).
static int run_contraction(pufe_ctx *ctx, const double *d_V, int precision, hipStream_t st, double *partial,
                           bool timed = true, const double *wimg = nullptr) {
    const bool saved = ctx->timing;
    ctx->timing = saved && timed;
    struct Restore {
        pufe_ctx *c;
        bool v;
        ~Restore() { c->timing = v; }
    } restore{ctx, saved};
    const Plan &pl = ctx->plan;
    KParams kp = pl.kp;
    kp.wimg = wimg;
    if (precision == PUFE_PREC_BF16X3 || precision == PUFE_PREC_BF16X6) {
        const int nl = precision == PUFE_PREC_BF16X3 ? 2 : 3;
        const size_t lds = split_lds_bytes(nl, ctx->max_rows_split, std::max(pl.max_nfun, 1), pl.max_img,
                                           ctx->max_item_leaves_split, pl.kp.n3);
        if (lds > kMaxDynLds) return fail(ctx, PUFE_ERR_UNSUPPORTED, "split stage does not fit in LDS");
        {
            TimedRegion tr(ctx, 0, st);
            CHECK_HIP(ctx, launch_contract_split(nl, pl.max_l, general_variant(pl), kp, (int)ctx->items_split.size(), ctx->d_items_split.p,
                                                 ctx->d_elems.p, ctx->d_groups.p, ctx->d_img.p, ctx->d_edof.p,
                                                 ctx->d_leaves.p, d_V, partial, lds, st),
                      "split contraction");
        }
    } else {
        TimedRegion tr(ctx, 0, st);
        // wide items first: they are the longest
        CHECK_HIP(ctx, launch_contract_wide(pl.max_l, general_variant(pl), kp, (int)ctx->items_wide.size(), ctx->d_items_wide.p,
                                            ctx->d_elems.p, ctx->d_groups.p, ctx->d_img.p, ctx->d_edof.p,
                                            ctx->d_leaves.p, d_V, partial, ctx->lds_wide, st),
                  "contraction (wide items)");
        CHECK_HIP(ctx, launch_contract_f64(ctx->contract_q, pl.max_l, general_variant(pl), kp, (int)ctx->items.size(), ctx->d_items.p,
                                           ctx->d_elems.p, ctx->d_groups.p, ctx->d_img.p, ctx->d_edof.p,
                                           ctx->d_leaves.p, d_V, partial, ctx->lds, st),
                  "contraction");
    }
    TimedRegion tr(ctx, 3, st);
    CHECK_HIP(ctx, launch_chunk_reduce(ctx->d_elems.p, ctx->d_reduce.p, (int)ctx->reduce.size(), partial, st),
              "K-chunk reduction");
    return PUFE_OK;
}

// Argument checks shared by pufe_assemble and pufe_assemble_noalloc.
static int check_assemble_args(pufe_ctx *ctx, const double *d_V, const double *kpts, int n_k, int precision,
                               int out_dtype, void *d_H) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "pufe_setup must come first");
    if (!d_V || !kpts || n_k < 1 || !d_H) return fail(ctx, PUFE_ERR_INVALID_ARG, "null pointer or n_k < 1");
    if (precision < PUFE_PREC_FP64 || precision > PUFE_PREC_BF16X6)
        return fail(ctx, PUFE_ERR_INVALID_ARG, "unknown precision");
    if (out_dtype < PUFE_OUT_C128 || out_dtype > PUFE_OUT_F64_GAMMA)
        return fail(ctx, PUFE_ERR_INVALID_ARG, "unknown output dtype");
    for (int k = 0; k < n_k; ++k) {
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(kpts[3 * k + d])) return fail(ctx, PUFE_ERR_INVALID_ARG, "non-finite k-point");
        if (out_dtype == PUFE_OUT_F64_GAMMA &&
            (std::fmod(kpts[3 * k], 1.0) != 0.0 || std::fmod(kpts[3 * k + 1], 1.0) != 0.0 ||
             std::fmod(kpts[3 * k + 2], 1.0) != 0.0))
            return fail(ctx, PUFE_ERR_INVALID_ARG, "real output needs every k-point at Gamma");
    }
    return PUFE_OK;
}

// Assembly with the Bloch-periodic enrichment: for every k-point the image
// weights, the contraction of the real and imaginary rows, the K-chunk sum,
// the projector coefficients of those rows (with projectors), the complex
// scatter of each colour into that k-point's output and the separable term.
static int assemble_bloch(pufe_ctx *ctx, const double *d_V, const double *kpts, int n_k, int precision,
                          int out_dtype, void *d_H, void *d_S, hipStream_t st, bool nonlocal) {
    const Plan &pl = ctx->plan;
    const int64_t per = out_dtype == PUFE_OUT_F64_GAMMA ? pl.nnz : 2 * pl.nnz;
    const size_t esz = out_dtype == PUFE_OUT_C64 ? sizeof(float) : sizeof(double);
    const int64_t nimg = (int64_t)(pl.img_nk.size() / 4);
    for (int k0 = 0; k0 < n_k; k0 += kMaxKPerLaunch) {
        KPoints kps;
        std::memset(&kps, 0, sizeof kps);
        kps.nk = std::min(kMaxKPerLaunch, n_k - k0);
        for (int k = 0; k < kps.nk; ++k)
            for (int d = 0; d < 3; ++d) kps.kap[k][d] = kpts[3 * (k0 + k) + d];
        {
            TimedRegion tr(ctx, 1, st);
            if (k0 == 0)
                CHECK_HIP(ctx, launch_prepare_outputs(d_H, d_S, (int64_t)(per * n_k * esz), kps, ctx->d_ztab.p, st),
                          "zero outputs and phase table");
            else
                CHECK_HIP(ctx, launch_phase_table(kps, ctx->d_ztab.p, st), "phase table");
        }
        for (int k = 0; k < kps.nk; ++k) {
            CHECK_HIP(ctx, launch_image_weights(ctx->d_img_nk.p, nimg, kps.kap[k], ctx->d_wimg.p, st),
                      "image weights");
            int rc = run_contraction(ctx, d_V, precision, st, ctx->d_partial.p, true, ctx->d_wimg.p);
            if (rc != PUFE_OK) return rc;
            const bool with_nl = nonlocal && pl.n_pfun > 0;
            if (with_nl) {
                // projector coefficients of this k-point's rows
                TimedRegion tn(ctx, 4, st);
                KParams kp = pl.kp;
                kp.wimg = ctx->d_wimg.p;
                CHECK_HIP(ctx, launch_nl_f(pl.max_l, kp, (int)ctx->nl_items.size(), ctx->d_nl_items.p, ctx->d_elems.p,
                                           ctx->d_groups.p, ctx->d_img.p, ctx->d_edof.p, ctx->d_leaves.p,
                                           ctx->d_pgroups.p, ctx->d_Fp.p, ctx->nl_lds, st),
                          "projector coefficients");
                CHECK_HIP(ctx, launch_nl_reduce(ctx->d_elems.p, ctx->d_nl_elems.p, (int)ctx->nl_elems.size(),
                                                ctx->d_Fp.p, st),
                          "projector coefficient sum");
            }
            TimedRegion tr(ctx, 1, st);
            char *H = (char *)d_H + (size_t)(k0 + k) * per * esz;
            char *S = d_S ? (char *)d_S + (size_t)(k0 + k) * per * esz : nullptr;
            for (size_t col = 0; col + 1 < pl.scat_off.size(); ++col) {
                const int n = (int)(pl.scat_off[col + 1] - pl.scat_off[col]);
                CHECK_HIP(ctx, launch_scatter_bloch(pl.kp, ctx->d_elems.p, ctx->d_scat.p + pl.scat_off[col], n,
                                                    ctx->d_edof.p, ctx->d_bpart.p, ctx->d_partial.p,
                                                    ctx->d_ztab.p + 27 * k, out_dtype, H, S, st),
                          "scatter");
            }
            if (with_nl) {
                // the separable term of this k-point into its H
                KPoints one;
                std::memset(&one, 0, sizeof one);
                one.nk = 1;
                for (int d = 0; d < 3; ++d) one.kap[0][d] = kps.kap[k][d];
                const int64_t ndof = pl.dof_off[pl.nv];
                CHECK_HIP(ctx, launch_nl_gather(pl.kp, ctx->d_elems.p, ctx->d_pgroups.p, ctx->d_edof.p, ctx->d_bpart.p,
                                                ctx->d_dof_el_off.p, ctx->d_dof_el.p, ctx->d_Fp.p, one, pl.n_pfun,
                                                ndof, ctx->d_nlf.p, st),
                          "projector sums");
                CHECK_HIP(ctx, launch_nl_update((int)pl.nl_blocks.size(), ctx->d_nl_blocks.p, ctx->d_brow.p,
                                                ctx->d_bcol.p, ctx->d_bval_off.p, ctx->d_dof_off.p, ctx->d_nlf.p,
                                                ctx->d_pfun_h.p, pl.n_pfun, ndof, 1, out_dtype, H, pl.nnz, st),
                          "nonlocal update");
            }
        }
    }
    return PUFE_OK;
}

// Contraction, K-chunk sum, output zero fill and coloured scatter of one
// assembly, with the partial tiles and the phase table in the given buffers.
static int assemble_impl(pufe_ctx *ctx, const double *d_V, const double *kpts, int n_k, int precision, int out_dtype,
                         void *d_H, void *d_S, hipStream_t st, double *partial, double2 *ztab, bool timed,
                         bool nonlocal = true) {
    if (ctx->plan.bloch) return assemble_bloch(ctx, d_V, kpts, n_k, precision, out_dtype, d_H, d_S, st, nonlocal);
    int rc = run_contraction(ctx, d_V, precision, st, partial, timed);
    if (rc != PUFE_OK) return rc;
    const Plan &pl = ctx->plan;
    const bool with_nl = nonlocal && pl.n_pfun > 0;
    if (with_nl) {
        // projector coefficients of every element a projector image reaches
        TimedRegion tn(ctx, timed ? 4 : -1, st);
        CHECK_HIP(ctx, launch_nl_f(pl.max_l, pl.kp, (int)ctx->nl_items.size(), ctx->d_nl_items.p, ctx->d_elems.p,
                                   ctx->d_groups.p, ctx->d_img.p, ctx->d_edof.p, ctx->d_leaves.p, ctx->d_pgroups.p,
                                   ctx->d_Fp.p, ctx->nl_lds, st),
                  "projector coefficients");
        CHECK_HIP(ctx, launch_nl_reduce(ctx->d_elems.p, ctx->d_nl_elems.p, (int)ctx->nl_elems.size(), ctx->d_Fp.p, st),
                  "projector coefficient sum");
    }
    TimedRegion tr(ctx, timed ? 1 : -1, st);
    const int64_t per = out_dtype == PUFE_OUT_F64_GAMMA ? pl.nnz : 2 * pl.nnz;
    const bool f32 = out_dtype == PUFE_OUT_C64;
    const size_t esz = f32 ? sizeof(float) : sizeof(double);
    for (int k0 = 0; k0 < n_k; k0 += kMaxKPerLaunch) {
        KPoints kps;
        std::memset(&kps, 0, sizeof kps);
        kps.nk = std::min(kMaxKPerLaunch, n_k - k0);
        for (int k = 0; k < kps.nk; ++k)
            for (int d = 0; d < 3; ++d) kps.kap[k][d] = kpts[3 * (k0 + k) + d];
        char *H = (char *)d_H + (size_t)k0 * per * esz;
        char *S = d_S ? (char *)d_S + (size_t)k0 * per * esz : nullptr;
        // the first pass zeroes every output (all k-points) with its phase table
        if (k0 == 0)
            CHECK_HIP(ctx, launch_prepare_outputs(d_H, d_S, (int64_t)(per * n_k * esz), kps, ztab, st),
                      "zero outputs and phase table");
        else
            CHECK_HIP(ctx, launch_phase_table(kps, ztab, st), "phase table");
        for (size_t col = 0; col + 1 < pl.scat_off.size(); ++col) {
            const int n = (int)(pl.scat_off[col + 1] - pl.scat_off[col]);
            CHECK_HIP(ctx, launch_scatter(pl.kp, ctx->d_elems.p, ctx->d_scat.p + pl.scat_off[col], n, ctx->d_edof.p,
                                          partial, ztab, kps.nk, out_dtype, H, S, pl.nnz, st),
                      "scatter");
        }
        if (with_nl) {
            // the separable term of these k-points into H
            const int64_t ndof = pl.dof_off[pl.nv];
            CHECK_HIP(ctx, launch_nl_gather(pl.kp, ctx->d_elems.p, ctx->d_pgroups.p, ctx->d_edof.p, nullptr,
                                            ctx->d_dof_el_off.p, ctx->d_dof_el.p, ctx->d_Fp.p, kps, pl.n_pfun, ndof,
                                            ctx->d_nlf.p, st),
                      "projector sums");
            CHECK_HIP(ctx, launch_nl_update((int)pl.nl_blocks.size(), ctx->d_nl_blocks.p, ctx->d_brow.p, ctx->d_bcol.p,
                                            ctx->d_bval_off.p, ctx->d_dof_off.p, ctx->d_nlf.p, ctx->d_pfun_h.p,
                                            pl.n_pfun, ndof, kps.nk, out_dtype, H, pl.nnz, st),
                      "nonlocal update");
        }
    }
    return PUFE_OK;
}

int pufe_assemble(pufe_ctx *ctx, const double *d_V, const double *kpts, int n_k, int precision, int out_dtype,
                  void *d_H, void *d_S, void *stream) {
    int rc = check_assemble_args(ctx, d_V, kpts, n_k, precision, out_dtype, d_H);
    if (rc != PUFE_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    return assemble_impl(ctx, d_V, kpts, n_k, precision, out_dtype, d_H, d_S, st, ctx->d_partial.p, ctx->d_ztab.p,
                         true);
}

int pufe_assemble_noalloc(pufe_ctx *ctx, const double *d_V, const double *kpts, int n_k, int precision, int out_dtype,
                          void *d_H, void *d_S, void *stream) {
    int rc = check_assemble_args(ctx, d_V, kpts, n_k, precision, out_dtype, d_H);
    if (rc != PUFE_OK) return rc;
    if (ctx->plan.n_pfun > 0)
        return fail(ctx, PUFE_ERR_UNSUPPORTED,
                    "pufe_assemble_noalloc: the nonlocal term keeps its coefficients in context buffers; use pufe_assemble");
    if (ctx->plan.bloch)
        return fail(ctx, PUFE_ERR_UNSUPPORTED,
                    "pufe_assemble_noalloc: the Bloch-periodic enrichment keeps its image weights in context buffers; "
                    "use pufe_assemble");
    // workspace: the phase table, then the partial tiles (256-byte aligned)
    const size_t ztab_bytes = (sizeof(double2) * kMaxKPerLaunch * 27 + 255) / 256 * 256;
    const size_t need = ztab_bytes + (size_t)ctx->part_slots * 512 * sizeof(double);
    if (need > kScratchBytes)
        return fail(ctx, PUFE_ERR_UNSUPPORTED,
                    "pufe_assemble_noalloc: this problem's partial tiles need " + std::to_string(need) +
                        " bytes of workspace, more than the fixed " + std::to_string(kScratchBytes) +
                        " bytes; use pufe_assemble");
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    double *ws = nullptr;
    CHECK_HIP(ctx, scratch_address(ctx->device, &ws), "workspace address");
    return assemble_impl(ctx, d_V, kpts, n_k, precision, out_dtype, d_H, d_S, st,
                         ws + ztab_bytes / sizeof(double), (double2 *)ws, false);
}

int pufe_element_matrices(pufe_ctx *ctx, int64_t elem, const double *d_V, int precision, double *d_He,
                          double *d_Se, int32_t *nloc, void *stream) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "pufe_setup must come first");
    if (!d_V || !d_He || !d_Se || elem < 0 || elem >= ctx->plan.nel)
        return fail(ctx, PUFE_ERR_INVALID_ARG, "bad element or null pointer");
    if (ctx->plan.bloch)
        return fail(ctx, PUFE_ERR_UNSUPPORTED, "element matrices of the Bloch-periodic enrichment are complex and per "
                                               "k-point; use pufe_assemble");
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    int rc = run_contraction(ctx, d_V, precision, st, ctx->d_partial.p);
    if (rc != PUFE_OK) return rc;
    CHECK_HIP(ctx, launch_elem_matrices(ctx->d_elems.p, elem, ctx->d_partial.p, d_He, d_Se, ctx->plan.elems[elem].nloc, st),
              "element matrices");
    if (nloc) *nloc = ctx->plan.elems[elem].nloc;
    return PUFE_OK;
}

// ------------------------------------------------ self-consistent field pieces

static bool dev_scalar(pufe_ctx *ctx, const double *d, double *h, hipStream_t st) {
    return hipMemcpyAsync(h, d, sizeof(double), hipMemcpyDeviceToHost, st) == hipSuccess &&
           hipStreamSynchronize(st) == hipSuccess;
}

// The (element, local function) pairs of every DOF and the per-element load
// sums, for the classical FE space's load vector.
static int ensure_fe_map(pufe_ctx *ctx, hipStream_t st) {
    const Plan &pl = ctx->plan;
    if (!ctx->d_dof_el_off.p) CHECK_HIP(ctx, ctx->d_dof_el_off.upload(pl.dof_el_off, st), "upload DOF map");
    if (!ctx->d_dof_el.p) CHECK_HIP(ctx, ctx->d_dof_el.upload(pl.dof_el, st), "upload DOF map");
    if (!ctx->d_fe_be.p) CHECK_HIP(ctx, ctx->d_fe_be.alloc((size_t)pl.nel * 32), "alloc load sums");
    return PUFE_OK;
}

static int fe_load_impl(pufe_ctx *ctx, const double *d_f, double *d_b, hipStream_t st) {
    const Plan &pl = ctx->plan;
    CHECK_HIP(ctx, launch_fe_load(pl.kp, ctx->d_elems.p, pl.nel, ctx->d_leaves.p, d_f, ctx->d_fe_be.p, pl.nv, pl.nfs,
                                  ctx->d_dof_off.p, ctx->d_dof_el_off.p, ctx->d_dof_el.p, d_b, st),
              "FE load vector");
    return PUFE_OK;
}

int pufe_fe_load(pufe_ctx *ctx, const double *d_f, double *d_b, void *stream) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "pufe_setup must come first");
    if (!d_f || !d_b) return fail(ctx, PUFE_ERR_INVALID_ARG, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    int rc = ensure_fe_map(ctx, st);
    if (rc != PUFE_OK) return rc;
    return fe_load_impl(ctx, d_f, d_b, st);
}

int pufe_fe_eval(pufe_ctx *ctx, const double *d_u, double *d_out, void *stream) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "pufe_setup must come first");
    if (!d_u || !d_out) return fail(ctx, PUFE_ERR_INVALID_ARG, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    CHECK_HIP(ctx, launch_fe_eval(ctx->plan.kp, ctx->d_elems.p, ctx->d_edof.p, ctx->d_leaves.p, ctx->d_leaf_elem.p,
                                  ctx->n_qp, d_u, d_out, st),
              "FE evaluation");
    return PUFE_OK;
}

// The Poisson operator of the classical FE space: K = 2 H restricted to the
// FE rows and columns of an assembly at Gamma with V = 0 (the kinetic term
// 1/2 int grad phi_i . grad phi_j of eq. disceig3d), without the separable
// term; and m_i = int phi_i.
static int build_poisson(pufe_ctx *ctx, hipStream_t st) {
    const Plan &pl = ctx->plan;
    const int64_t nfe = pl.nv * pl.nfs, nnzb = (int64_t)pl.bcol.size();
    {
        DevBuf<double> zeroV, Hfull;
        CHECK_HIP(ctx, zeroV.alloc((size_t)std::max<int64_t>(ctx->n_qp, 1)), "alloc zero potential");
        CHECK_HIP(ctx, launch_fill_zero(zeroV.p, ctx->n_qp, false, st), "zero potential");
        CHECK_HIP(ctx, Hfull.alloc((size_t)pl.nnz), "alloc kinetic matrix");
        const double gamma[3] = {0.0, 0.0, 0.0};
        int rc = assemble_impl(ctx, zeroV.p, gamma, 1, PUFE_PREC_FP64, PUFE_OUT_F64_GAMMA, Hfull.p, nullptr, st,
                               ctx->d_partial.p, ctx->d_ztab.p, false, false);
        if (rc != PUFE_OK) return rc;
        CHECK_HIP(ctx, ctx->d_Kfe.alloc((size_t)(nnzb * pl.nfs * pl.nfs)), "alloc FE stiffness");
        CHECK_HIP(ctx, launch_fe_blocks(nnzb, pl.nfs, ctx->d_bcol.p, ctx->d_bval_off.p, ctx->d_dof_off.p, Hfull.p, 2.0,
                                        ctx->d_Kfe.p, st),
                  "FE stiffness blocks");
        CHECK_HIP(ctx, hipStreamSynchronize(st), "sync");
    }
    CHECK_HIP(ctx, ctx->d_brow_ptr.upload(pl.brow_ptr, st), "upload block rows");
    CHECK_HIP(ctx, ctx->d_mfe.alloc((size_t)nfe), "alloc FE integrals");
    CHECK_HIP(ctx, ctx->d_fe_ones.alloc((size_t)std::max<int64_t>(nfe, ctx->n_qp)), "alloc ones");
    {
        std::vector<double> ones((size_t)std::max<int64_t>(nfe, ctx->n_qp), 1.0);
        CHECK_HIP(ctx, ctx->d_fe_ones.upload(ones, st), "upload ones");
    }
    int rc = fe_load_impl(ctx, ctx->d_fe_ones.p, ctx->d_mfe.p, st);
    if (rc != PUFE_OK) return rc;
    CHECK_HIP(ctx, ctx->d_cg.alloc((size_t)(5 * nfe)), "alloc CG workspace");
    CHECK_HIP(ctx, ctx->d_dot.alloc((size_t)(dot_partial_slots() + 1)), "alloc dot workspace");
    double *out = ctx->d_dot.p + dot_partial_slots();
    CHECK_HIP(ctx, launch_dot(nfe, ctx->d_mfe.p, ctx->d_fe_ones.p, ctx->d_dot.p, out, st), "dot");
    if (!dev_scalar(ctx, out, &ctx->m_sum, st)) return fail(ctx, PUFE_ERR_HIP, "read FE integral sum");
    ctx->have_poisson = true;
    return PUFE_OK;
}

int pufe_hartree(pufe_ctx *ctx, const double *d_n, double *d_vh, double *d_v, double tol, int max_iter,
                 int *iters, double *resid, void *stream) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "pufe_setup must come first");
    if (!d_n || !d_vh) return fail(ctx, PUFE_ERR_INVALID_ARG, "null pointer");
    if (!(tol > 0.0) || max_iter < 1) return fail(ctx, PUFE_ERR_INVALID_ARG, "need tol > 0 and max_iter >= 1");
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    int rc = ensure_fe_map(ctx, st);
    if (rc != PUFE_OK) return rc;
    if (!ctx->have_poisson) {
        rc = build_poisson(ctx, st);
        if (rc != PUFE_OK) return rc;
    }
    const Plan &pl = ctx->plan;
    const int64_t n = pl.nv * pl.nfs;
    double *b = ctx->d_cg.p, *r = b + n, *p = r + n, *Ap = p + n, *x = Ap + n;
    double *part = ctx->d_dot.p, *out = part + dot_partial_slots();
    auto dot = [&](const double *a, const double *c, double *h) -> int {
        CHECK_HIP(ctx, launch_dot(n, a, c, part, out, st), "dot");
        if (!dev_scalar(ctx, out, h, st)) return fail(ctx, PUFE_ERR_HIP, "read dot product");
        return PUFE_OK;
    };
    // right-hand side 4 pi (b - nbar m), nbar = int n / int 1 (the neutralising background)
    rc = fe_load_impl(ctx, d_n, b, st);
    if (rc != PUFE_OK) return rc;
    double bsum = 0.0;
    if ((rc = dot(b, ctx->d_fe_ones.p, &bsum)) != PUFE_OK) return rc;
    const double nbar = bsum / ctx->m_sum;
    CHECK_HIP(ctx, launch_scaled_diff(n, 4.0 * M_PI, b, nbar, ctx->d_mfe.p, r, st), "right-hand side");
    // conjugate gradients on K x = r from x = 0 (K is singular with the
    // constants as its kernel; r is orthogonal to them)
    CHECK_HIP(ctx, launch_fill_zero(x, n, false, st), "zero solution");
    CHECK_HIP(ctx, hipMemcpyAsync(p, r, sizeof(double) * n, hipMemcpyDeviceToDevice, st), "copy residual");
    double rr = 0.0;
    if ((rc = dot(r, r, &rr)) != PUFE_OK) return rc;
    const double r0 = std::sqrt(rr);
    int it = 0;
    double rel = 0.0;
    if (r0 > 0.0) {
        for (; it < max_iter; ++it) {
            CHECK_HIP(ctx, launch_fe_spmv(pl.nv, pl.nfs, ctx->d_brow_ptr.p, ctx->d_bcol.p, ctx->d_Kfe.p, p, Ap, st),
                      "FE stiffness product");
            double pAp = 0.0;
            if ((rc = dot(p, Ap, &pAp)) != PUFE_OK) return rc;
            if (!(pAp > 0.0)) break;
            const double alpha = rr / pAp;
            CHECK_HIP(ctx, launch_axpby(n, alpha, p, 1.0, x, st), "CG update");
            CHECK_HIP(ctx, launch_axpby(n, -alpha, Ap, 1.0, r, st), "CG update");
            double rn = 0.0;
            if ((rc = dot(r, r, &rn)) != PUFE_OK) return rc;
            rel = std::sqrt(rn) / r0;
            if (rel <= tol) {
                ++it;
                break;
            }
            CHECK_HIP(ctx, launch_axpby(n, 1.0, r, rn / rr, p, st), "CG direction");
            rr = rn;
        }
    }
    // zero mean: int V_H = sum_i x_i m_i = 0
    double mx = 0.0;
    if ((rc = dot(ctx->d_mfe.p, x, &mx)) != PUFE_OK) return rc;
    CHECK_HIP(ctx, launch_axpby(n, -mx / ctx->m_sum, ctx->d_fe_ones.p, 1.0, x, st), "zero mean");
    if (d_v) CHECK_HIP(ctx, hipMemcpyAsync(d_v, x, sizeof(double) * n, hipMemcpyDeviceToDevice, st), "copy solution");
    CHECK_HIP(ctx, launch_fe_eval(pl.kp, ctx->d_elems.p, ctx->d_edof.p, ctx->d_leaves.p, ctx->d_leaf_elem.p,
                                  ctx->n_qp, x, d_vh, st),
              "Hartree potential at the points");
    if (iters) *iters = it;
    if (resid) *resid = rel;
    return PUFE_OK;
}

int pufe_lda_xc(int64_t n, const double *d_rho, double *d_vxc, double *d_exc, void *stream) {
    if (n < 0 || (n > 0 && (!d_rho || !d_vxc))) return PUFE_ERR_INVALID_ARG;
    hipError_t e = launch_lda_xc(n, d_rho, d_vxc, d_exc, (hipStream_t)stream);
    return e == hipSuccess ? PUFE_OK : PUFE_ERR_HIP;
}

// Plan the adjoint: one work item per (element, K-chunk of the forward
// partition), the padded Ps blocks, and for each atom the list of per-item
// group partial forces in a fixed order.
static int plan_backward(pufe_ctx *c, hipStream_t st) {
    Plan &pl = c->plan;
    int max_npad = 16, max_nfun = 1, max_nenr = 1, max_nfun_wide = 1;
    std::vector<int64_t> pt_off(pl.nel + 1, 0);
    // an element runs the block-resident kernel when it has at most 80
    // functions and the launch's stage (sized by the largest Ps, row count and
    // enrichment table of its elements) still fits in LDS with it: elements
    // are taken in order of their own stage size; the others run the wide
    // kernel
    const int nimg = std::max(pl.max_img, 1);
    std::vector<char> wide(pl.nel, 1);
    {
        std::vector<std::pair<size_t, int64_t>> order;
        for (int64_t e = 0; e < pl.nel; ++e) {
            const ElemDev &el = pl.elems[e];
            if (el.nloc <= kBackwardMaxNloc)
                order.push_back({backward_lds_bytes(16 * ((el.nloc + 15) / 16), el.nloc - el.nfe, el.nfun, nimg), e});
        }
        std::stable_sort(order.begin(), order.end());
        int np = 16, ne = 1, nf = 1;
        for (const auto &o : order) {
            const ElemDev &el = pl.elems[o.second];
            const int np2 = std::max(np, 16 * ((el.nloc + 15) / 16)), ne2 = std::max(ne, el.nloc - el.nfe);
            const int nf2 = std::max(nf, el.nfun);
            if (backward_lds_bytes(np2, ne2, nf2, nimg) > kMaxDynLds) continue;
            np = np2, ne = ne2, nf = nf2;
            wide[o.second] = 0;
        }
    }
    for (int64_t e = 0; e < pl.nel; ++e) {
        const ElemDev &el = pl.elems[e];
        const int npad = 16 * ((el.nloc + 15) / 16);
        if (wide[e]) {
            if (el.nloc - el.nfe > kBackwardWideMaxEnr)
                return fail(c, PUFE_ERR_UNSUPPORTED, "the adjoint kernels hold at most " +
                                                         std::to_string(kBackwardWideMaxEnr) +
                                                         " enriched functions on one element");
            max_nfun_wide = std::max(max_nfun_wide, el.nfun);
        } else {
            max_npad = std::max(max_npad, npad);
            max_nfun = std::max(max_nfun, el.nfun);
            max_nenr = std::max(max_nenr, el.nloc - el.nfe);
        }
        pt_off[e + 1] = pt_off[e] + (int64_t)npad * npad;
    }
    c->bw_lds = backward_lds_bytes(max_npad, max_nenr, max_nfun, nimg);
    c->bw_lds_wide = backward_wide_lds_bytes(max_nfun_wide, nimg);
    if (c->bw_lds > kMaxDynLds || c->bw_lds_wide > kMaxDynLds)
        return fail(c, PUFE_ERR_UNSUPPORTED, "adjoint stage does not fit in LDS");
    c->bw_items.clear();
    c->bw_items_wide.clear();
    const int mg = std::max(pl.max_ngrp, 1);
    // items of elements up to 80 functions first, then the wide ones; the
    // partial-force slots follow that order
    for (int pass = 0; pass < 2; ++pass)
        for (int64_t e = 0; e < pl.nel; ++e) {
            const ElemDev &el = pl.elems[e];
            if ((wide[e] != 0) != (pass == 1)) continue;
            // twice the forward's K-chunks (at most one per leaf): the adjoint's
            // stages cost more, and finer items balance the refined elements
            int64_t nleaf = el.leaf_end - el.leaf_off, nch = std::min<int64_t>(2 * el.nchunk, nleaf);
            for (int64_t ch = 0; ch < nch; ++ch) {
                ItemDev it{};
                it.elem = (int32_t)e;
                it.chunk = (int32_t)ch;
                it.leaf_b = el.leaf_off + ch * nleaf / nch;
                it.leaf_e = el.leaf_off + (ch + 1) * nleaf / nch;
                (pass == 0 ? c->bw_items : c->bw_items_wide).push_back(it);
            }
        }
    std::vector<std::vector<int64_t>> slots(c->prob.species.size());
    const int64_t nn = (int64_t)c->bw_items.size(), ntot = nn + (int64_t)c->bw_items_wide.size();
    for (int64_t idx = 0; idx < ntot; ++idx) {
        const ItemDev &it = idx < nn ? c->bw_items[idx] : c->bw_items_wide[idx - nn];
        const ElemDev &el = pl.elems[it.elem];
        for (int g = 0; g < el.ngrp; ++g) slots[pl.groups[el.grp_off + g].atom].push_back(idx * mg + g);
    }
    std::vector<int64_t> aptr(slots.size() + 1, 0), aslots;
    for (size_t A = 0; A < slots.size(); ++A) {
        aslots.insert(aslots.end(), slots[A].begin(), slots[A].end());
        aptr[A + 1] = (int64_t)aslots.size();
    }
    CHECK_HIP(c, c->d_bw_items.upload(c->bw_items, st), "upload adjoint items");
    CHECK_HIP(c, c->d_bw_items_wide.upload(c->bw_items_wide, st), "upload adjoint items");
    CHECK_HIP(c, c->d_pt_off.upload(pt_off, st), "upload adjoint offsets");
    CHECK_HIP(c, c->d_atom_ptr.upload(aptr, st), "upload atom lists");
    CHECK_HIP(c, c->d_atom_slots.upload(aslots, st), "upload atom lists");
    CHECK_HIP(c, c->d_Pt.alloc((size_t)pt_off[pl.nel]), "alloc adjoint blocks");
    CHECK_HIP(c, c->d_fP.alloc((size_t)ntot * mg * 3), "alloc partial forces");
    CHECK_HIP(c, c->d_fQ.alloc((size_t)ntot * mg * 3), "alloc partial forces");
    c->have_bw = true;
    return PUFE_OK;
}

int pufe_assemble_backward(pufe_ctx *ctx, const double *d_V, const double kpt[3], const void *d_P, const void *d_Q,
                           int precision, double *d_dLdV, double *d_dLdR, void *stream) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "pufe_setup must come first");
    if (!d_V || !kpt) return fail(ctx, PUFE_ERR_INVALID_ARG, "null V or k-point");
    if (precision < PUFE_PREC_FP64 || precision > PUFE_PREC_BF16X6)
        return fail(ctx, PUFE_ERR_INVALID_ARG, "unknown precision");
    const int nl = precision == PUFE_PREC_BF16X3 ? 2 : (precision == PUFE_PREC_BF16X6 ? 3 : 0);
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(kpt[d])) return fail(ctx, PUFE_ERR_INVALID_ARG, "non-finite k-point");
    if (ctx->plan.bloch)
        return fail(ctx, PUFE_ERR_UNSUPPORTED, "the adjoint of the Bloch-periodic enrichment is not supported");
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (!ctx->have_bw) {
        int rc = plan_backward(ctx, st);
        if (rc != PUFE_OK) return rc;
    }
    const Plan &pl = ctx->plan;
    const int nwide = (int)ctx->bw_items_wide.size();
    if (nl != 0 && nwide > 0)
        return fail(ctx, PUFE_ERR_UNSUPPORTED,
                    "the split-precision adjoint holds elements of at most " + std::to_string(kBackwardMaxNloc) +
                        " functions (use FP64)");
    TimedRegion tr(ctx, 2, st);
    const int mg = std::max(pl.max_ngrp, 1);
    const int nit = (int)ctx->bw_items.size();
    const size_t wide_slots = (size_t)nit * mg * 3;   // the wide items' partial forces follow the others
    if (d_P) {
        CHECK_HIP(ctx, launch_gather_adjoint(pl.kp, pl.nel, ctx->d_elems.p, ctx->d_edof.p, ctx->d_pt_off.p,
                                             (const double *)d_P, kpt, ctx->d_Pt.p, st), "gather P");
        CHECK_HIP(ctx, launch_backward(pl.kp, false, nl, nit, ctx->d_bw_items.p, ctx->d_elems.p, ctx->d_groups.p,
                                       ctx->d_img.p, ctx->d_edof.p, ctx->d_leaves.p, d_V, ctx->d_pt_off.p,
                                       ctx->d_Pt.p, d_dLdV, ctx->d_fP.p, mg, ctx->bw_lds, st), "adjoint (P)");
        CHECK_HIP(ctx, launch_backward_wide(pl.kp, false, nwide, ctx->d_bw_items_wide.p, ctx->d_elems.p,
                                            ctx->d_groups.p, ctx->d_img.p, ctx->d_edof.p, ctx->d_leaves.p, d_V,
                                            ctx->d_pt_off.p, ctx->d_Pt.p, d_dLdV, ctx->d_fP.p + wide_slots, mg,
                                            ctx->bw_lds_wide, st), "adjoint (P, wide elements)");
    } else if (d_dLdV) {
        CHECK_HIP(ctx, launch_fill_zero(d_dLdV, ctx->n_qp, false, st), "zero dLdV");
    }
    if (d_Q) {
        CHECK_HIP(ctx, launch_gather_adjoint(pl.kp, pl.nel, ctx->d_elems.p, ctx->d_edof.p, ctx->d_pt_off.p,
                                             (const double *)d_Q, kpt, ctx->d_Pt.p, st), "gather Q");
        CHECK_HIP(ctx, launch_backward(pl.kp, true, nl, nit, ctx->d_bw_items.p, ctx->d_elems.p, ctx->d_groups.p,
                                       ctx->d_img.p, ctx->d_edof.p, ctx->d_leaves.p, d_V, ctx->d_pt_off.p,
                                       ctx->d_Pt.p, nullptr, ctx->d_fQ.p, mg, ctx->bw_lds, st), "adjoint (Q)");
        CHECK_HIP(ctx, launch_backward_wide(pl.kp, true, nwide, ctx->d_bw_items_wide.p, ctx->d_elems.p,
                                            ctx->d_groups.p, ctx->d_img.p, ctx->d_edof.p, ctx->d_leaves.p, d_V,
                                            ctx->d_pt_off.p, ctx->d_Pt.p, nullptr, ctx->d_fQ.p + wide_slots, mg,
                                            ctx->bw_lds_wide, st), "adjoint (Q, wide elements)");
    }
    if (d_dLdR)
        CHECK_HIP(ctx, launch_force_reduce((int)ctx->prob.species.size(), ctx->d_atom_ptr.p, ctx->d_atom_slots.p,
                                           d_P ? ctx->d_fP.p : nullptr, d_Q ? ctx->d_fQ.p : nullptr, d_dLdR, st),
                  "force reduction");
    return PUFE_OK;
}

int pufe_set_positions(pufe_ctx *ctx, const double *pos) {
    if (!ctx || !pos) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_problem) return fail(ctx, PUFE_ERR_STATE, "no problem defined");
    Plan &pl = ctx->plan;
    const size_t na = ctx->prob.species.size();
    for (size_t A = 0; A < na; ++A) {
        double d2 = 0;
        for (int c = 0; c < 3; ++c) {
            if (!std::isfinite(pos[3 * A + c])) return fail(ctx, PUFE_ERR_INVALID_ARG, "non-finite position");
            double d = pos[3 * A + c] - ctx->prob.pos[3 * A + c];
            d2 += d * d;
        }
        if (std::sqrt(d2) > kImageMargin)
            return fail(ctx, PUFE_ERR_INVALID_ARG, "an enrichment centre moved farther than the image margin");
    }
    // shift every image centre of a group by its atom's displacement
    for (const ElemDev &el : pl.elems)
        for (int g = 0; g < el.ngrp; ++g) {
            const GroupDev &G = pl.groups[el.grp_off + g];
            for (int k = 0; k < G.nimg; ++k)
                for (int c = 0; c < 3; ++c)
                    pl.img_cur[3 * (G.img_off + k) + c] = pl.img[3 * (G.img_off + k) + c] +
                                                          (pos[3 * G.atom + c] - ctx->prob.pos[3 * G.atom + c]);
        }
    if (ctx->have_setup) {
        CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        CHECK_HIP(ctx, hipMemcpy(ctx->d_img.p, pl.img_cur.data(), sizeof(double) * pl.img_cur.size(),
                                 hipMemcpyHostToDevice), "upload image centres");
    }
    return PUFE_OK;
}

int pufe_bsr_to_dense(pufe_ctx *ctx, const void *d_bsr, int dtype, double *d_dense, void *stream) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "pufe_setup must come first");
    if (!d_bsr || !d_dense) return fail(ctx, PUFE_ERR_INVALID_ARG, "null pointer");
    if (dtype != PUFE_OUT_C128 && dtype != PUFE_OUT_F64_GAMMA)
        return fail(ctx, PUFE_ERR_INVALID_ARG, "dense expansion takes C128 or F64_GAMMA values");
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    const Plan &pl = ctx->plan;
    int64_t n = pl.dof_off[pl.nv];
    CHECK_HIP(ctx, launch_fill_zero(d_dense, 2 * n * n, false, st), "zero dense");
    CHECK_HIP(ctx, launch_bsr_to_dense((int64_t)pl.bcol.size(), ctx->d_brow.p, ctx->d_bcol.p, ctx->d_bval_off.p,
                                       ctx->d_dof_off.p, d_bsr, dtype == PUFE_OUT_C128 ? 0 : 1, n, d_dense, st),
              "bsr to dense");
    return PUFE_OK;
}

int pufe_enable_timing(pufe_ctx *ctx, int on) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    ctx->timing = on != 0;
    return PUFE_OK;
}

int pufe_kernel_times(pufe_ctx *ctx, double *out_ms, int64_t *counts, int reset) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    for (int k = 0; k < 5; ++k) {
        double ms = 0.0;
        for (auto &pr : ctx->ev[k]) {
            CHECK_HIP(ctx, hipEventSynchronize(pr.second), "event sync");
            float t = 0.f;
            CHECK_HIP(ctx, hipEventElapsedTime(&t, pr.first, pr.second), "event time");
            ms += t;
        }
        if (out_ms) out_ms[k] = ms;
        if (counts) counts[k] = (int64_t)ctx->ev[k].size();
    }
    if (reset) ctx->clear_events();
    return PUFE_OK;
}

// Upload the element table, work items and partial buffer of the current plan.
static int upload_items(pufe_ctx *ctx, hipStream_t st) {
    ++ctx->plan_gen;
    CHECK_HIP(ctx, ctx->d_elems.upload(ctx->plan.elems, st), "upload elements");
    CHECK_HIP(ctx, ctx->d_items.upload(ctx->items, st), "upload work items");
    CHECK_HIP(ctx, ctx->d_items_wide.upload(ctx->items_wide, st), "upload work items");
    CHECK_HIP(ctx, ctx->d_items_split.upload(ctx->items_split, st), "upload work items");
    CHECK_HIP(ctx, ctx->d_reduce.upload(ctx->reduce, st), "upload chunk reduction list");
    CHECK_HIP(ctx, ctx->d_partial.alloc((size_t)ctx->part_slots * 512), "alloc partial tiles");
    ctx->have_bw = false;
    ctx->have_poisson = false;
    return upload_nonlocal(ctx, st);
}

int pufe_tune(pufe_ctx *ctx, int precision, const char *cache_path) {
    if (!ctx) return PUFE_ERR_INVALID_ARG;
    if (!ctx->have_setup) return fail(ctx, PUFE_ERR_STATE, "pufe_setup must come first");
    if (precision < PUFE_PREC_FP64 || precision > PUFE_PREC_BF16X6)
        return fail(ctx, PUFE_ERR_INVALID_ARG, "unknown precision");
    CHECK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    const Plan &pl = ctx->plan;
    int64_t sum_nloc = 0;
    for (const ElemDev &el : pl.elems) sum_nloc += el.nloc;
    char key[256];
    hipDeviceProp_t prop;
    CHECK_HIP(ctx, hipGetDeviceProperties(&prop, ctx->device), "device properties");
    std::snprintf(key, sizeof key, "%s|prec%d|nel%lld|leaves%lld|n3_%d|nloc%lld|maxnloc%d", prop.gcnArchName, precision,
                  (long long)pl.nel, (long long)ctx->n_leaves, pl.kp.n3, (long long)sum_nloc, pl.max_nloc);
    // cached choice?
    std::string text;
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "rb")) {
            char buf[4096];
            size_t r;
            while ((r = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, r);
            std::fclose(f);
        }
        std::string pat = std::string("\"") + key + "\": {\"items\": ";
        size_t at = text.find(pat);
        if (at != std::string::npos) {
            double items = 0;
            int block = 0, qv = 0, wide = kWideTiles;
            const int nf = std::sscanf(text.c_str() + at + pat.size(), "%lf, \"block\": %d, \"q\": %d, \"wide\": %d",
                                       &items, &block, &qv, &wide);
            if (nf >= 3 && items > 0 && block >= 1 && block <= kBlockTiles && contract_q_supported(qv) &&
                (wide == 0 || (wide >= 2 && wide <= kWideTiles))) {
                ctx->tune_items = items;
                ctx->tune_block = block;
                ctx->contract_q = qv;
                ctx->wide_tiles = wide;
                ctx->tuned = true;
                plan_items(ctx, items, block);
                return upload_items(ctx, nullptr);
            }
        }
    }
    DevBuf<double> V;
    CHECK_HIP(ctx, V.alloc(std::max<int64_t>(ctx->n_qp, 1)), "alloc timing input");
    CHECK_HIP(ctx, hipMemset(V.p, 0, sizeof(double) * V.n), "zero timing input");
    hipEvent_t a, b;
    CHECK_HIP(ctx, hipEventCreate(&a), "event");
    CHECK_HIP(ctx, hipEventCreate(&b), "event");
    const bool saved = ctx->timing;
    ctx->timing = false;
    // Coordinate descent from the current choice: the item count first, then
    // the tile block, then the stage length, each candidate timed once after
    // a warm-up run (a problem of a few hundred milliseconds per assembly is
    // tuned in seconds rather than minutes).
    double best = 1e300, best_items = ctx->tune_items;
    int best_block = ctx->tune_block, best_q = ctx->contract_q, best_wide = ctx->wide_tiles;
    struct Tried {
        double items;
        int block, q, wide;
    };
    std::vector<Tried> tried;
    auto trial = [&](double items, int block, int qv, int wide) -> int {
        for (auto &t : tried)
            if (t.items == items && t.block == block && t.q == qv && t.wide == wide) return PUFE_OK;
        tried.push_back({items, block, qv, wide});
        ctx->contract_q = qv;
        ctx->wide_tiles = wide;
        plan_items(ctx, items, block);
        if (ctx->lds > kMaxDynLds || ctx->contract_q != qv) return PUFE_OK;   // does not fit: skip
        int rc = upload_items(ctx, nullptr);
        if (rc != PUFE_OK) return rc;
        rc = run_contraction(ctx, V.p, precision, nullptr, ctx->d_partial.p);   // warm-up
        if (rc != PUFE_OK) return rc;
        CHECK_HIP(ctx, hipEventRecord(a, nullptr), "event");
        rc = run_contraction(ctx, V.p, precision, nullptr, ctx->d_partial.p);
        if (rc != PUFE_OK) return rc;
        CHECK_HIP(ctx, hipEventRecord(b, nullptr), "event");
        CHECK_HIP(ctx, hipEventSynchronize(b), "event");
        float ms = 0;
        CHECK_HIP(ctx, hipEventElapsedTime(&ms, a, b), "event");
        if (ms < best) {
            best = ms;
            best_items = items;
            best_block = block;
            best_q = qv;
            best_wide = wide;
        }
        return PUFE_OK;
    };
    int trc = PUFE_OK;
    const int start_block = ctx->tune_block, start_q = ctx->contract_q, start_wide = ctx->wide_tiles;
    for (double items : {1024.0, 2048.0, 4096.0, 8192.0, 16384.0})
        if (trc == PUFE_OK) trc = trial(items, start_block, start_q, start_wide);
    for (int block = 2; block <= kBlockTiles && trc == PUFE_OK; ++block)
        trc = trial(best_items, block, start_q, start_wide);
    for (int qv : {16, 24, 32})
        if (trc == PUFE_OK) trc = trial(best_items, best_block, qv, start_wide);
    if (pl.max_nloc > 16 * kWholeMaxTiles)   // elements for the wide kernel
        for (int wide : {kWideTiles, kWideTiles - 1, 0})
            if (trc == PUFE_OK) trc = trial(best_items, best_block, best_q, wide);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (trc != PUFE_OK) {
        ctx->timing = saved;
        return trc;
    }
    ctx->timing = saved;
    ctx->tune_items = best_items;
    ctx->tune_block = best_block;
    ctx->contract_q = best_q;
    ctx->wide_tiles = best_wide;
    ctx->tuned = true;
    plan_items(ctx, best_items, best_block);
    int rc = upload_items(ctx, nullptr);
    if (rc != PUFE_OK) return rc;
    if (cache_path) {
        // append or insert the entry into a flat JSON object
        char entry[512];
        std::snprintf(entry, sizeof entry, "\"%s\": {\"items\": %.0f, \"block\": %d, \"q\": %d, \"wide\": %d, \"ms\": %.4f}",
                      key, best_items, best_block, best_q, best_wide, best);
        size_t close = text.rfind('}');
        std::string out;
        if (close == std::string::npos || text.find('{') == std::string::npos)
            out = std::string("{\n  ") + entry + "\n}\n";
        else {
            std::string head = text.substr(0, close);
            while (!head.empty() && (head.back() == '\n' || head.back() == ' ')) head.pop_back();
            out = head + (head.back() == '{' ? "\n  " : ",\n  ") + entry + "\n}\n";
        }
        if (FILE *f = std::fopen(cache_path, "wb")) {
            std::fwrite(out.data(), 1, out.size(), f);
            std::fclose(f);
        }
    }
    return PUFE_OK;
}

// stage lengths of the batch's FP64 classes, longest first; each has a class
// of problems sharing a CU two work groups at a time and one of the rest
static const int kBatchQ[3] = {32, 24, 16};
constexpr int kBatchClasses = 6;

struct pufe_batch {
    std::vector<pufe_ctx *> ctxs;
    std::vector<uint64_t> gens;             // plan generation of each context at creation
    int device = 0;
    std::vector<ItemDev> items, items_split;
    std::vector<std::vector<int4>> lists;   // per colour: (problem, element, tile pair)
    // FP64 items in up to kBatchClasses classes, each a persistent launch of
    // its own (items [item_off[c], item_off[c + 1])): per stage length, the
    // problems whose combined stage fits two work groups per CU, then the rest
    size_t lds_f64[kBatchClasses] = {}, lds_split[2] = {0, 0};
    int max_l = 0, q[kBatchClasses] = {};
    bool gen = false;                       // some problem needs the general kernel variant
    int grid_f64[kBatchClasses] = {}, grid_split[2] = {0, 0};
    int64_t item_off[kBatchClasses + 1] = {};
    // wide items of all problems (8-wave persistent launch)
    std::vector<ItemDev> items_wide;
    size_t lds_wide = 0;
    int grid_wide = 0;
    DevBuf<CtxDev> d_ctxs;
    DevBuf<ItemDev> d_items, d_items_split, d_items_wide;
    DevBuf<int4> d_lists;
    std::vector<int4> reduce;               // (problem, element, tile pair) of multi-chunk elements
    DevBuf<int4> d_reduce;
    DevBuf<double2> d_ztab;
    std::vector<int64_t> list_off;
    DevBuf<int> d_counter;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uintptr_t> key;
    std::string err;
    ~pufe_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

static int bfail(pufe_batch *b, int code, const std::string &msg) {
    if (b) b->err = msg;
    return code;
}

#define CHECK_HIP_B(b, x, where)                                                               \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess)                                                                  \
            return bfail(b, e_ == hipErrorOutOfMemory ? PUFE_ERR_OOM : PUFE_ERR_HIP,            \
                         std::string(where) + ": " + hipGetErrorString(e_));                   \
    } while (0)

static double item_cost(const ItemDev &it, int n3) {
    const int pairs = it.I0 == it.J0 ? it.nI * (it.nI + 1) / 2 : it.nI * it.nJ;
    return (double)pairs * (double)(it.leaf_e - it.leaf_b) * n3;
}

int pufe_batch_create(pufe_batch **out, pufe_ctx *const *ctxs, int n) {
    if (!out || !ctxs || n < 1) return PUFE_ERR_INVALID_ARG;
    pufe_batch *b = new (std::nothrow) pufe_batch();
    if (!b) return PUFE_ERR_OOM;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i] || !ctxs[i]->have_setup || ctxs[i]->device != ctxs[0]->device) {
            delete b;
            return PUFE_ERR_STATE;
        }
        if (ctxs[i]->plan.n_pfun > 0 || ctxs[i]->plan.bloch) {   // no nonlocal or per-k launches in the batch graph
            delete b;
            return PUFE_ERR_UNSUPPORTED;
        }
        b->ctxs.push_back(ctxs[i]);
        b->gens.push_back(ctxs[i]->plan_gen);
    }
    b->device = ctxs[0]->device;
    if (hipSetDevice(b->device) != hipSuccess) { delete b; return PUFE_ERR_HIP; }
    int max_rows_split = 16, max_nfun = 1, max_img = 0, max_leaves_split = 1, max_n3 = 1;
    b->lists.assign(27, {});
    // FP64 classes.  Each problem keeps its own stage length (the one pufe_tune
    // chose, else the library default); the problems of one length, in order of
    // their own stage size, join that length's first class while the class's
    // combined stage still fits two work groups per CU, the others its second.
    std::vector<int> cls(n, 0);
    for (int qi = 0; qi < 3; ++qi) {
        const int qv = kBatchQ[qi];
        std::vector<std::pair<size_t, int>> by_lds;
        for (int i = 0; i < n; ++i) {
            const pufe_ctx *c = ctxs[i];
            const int qc = contract_q_supported(c->contract_q) ? c->contract_q : 24;
            if (qc != qv) continue;
            by_lds.push_back({contract_lds_bytes(qv, c->max_rows, std::max(c->plan.max_nfun, 1), c->plan.max_img,
                                                 c->max_item_leaves, c->plan.kp.n3), i});
        }
        std::stable_sort(by_lds.begin(), by_lds.end());
        int r = 16, f = 1, im = 0, lv = 1, n3 = 1;
        for (const auto &pr : by_lds) {
            const pufe_ctx *c = ctxs[pr.second];
            const int r2 = std::max(r, c->max_rows), f2 = std::max(f, c->plan.max_nfun), im2 = std::max(im, c->plan.max_img);
            const int lv2 = std::max(lv, c->max_item_leaves), n32 = std::max(n3, c->plan.kp.n3);
            cls[pr.second] = 2 * qi + 1;
            if (persistent_blocks_per_cu(contract_lds_bytes(qv, r2, f2, im2, lv2, n32)) < 2) continue;
            r = r2, f = f2, im = im2, lv = lv2, n3 = n32;
            cls[pr.second] = 2 * qi;
        }
    }
    for (int pass = 0; pass < kBatchClasses + 2; ++pass) {
        // passes 0 .. kBatchClasses-1: FP64 items of each class; then the
        // split items and the wide FP64 items
        const int split_pass = kBatchClasses, wide_pass = kBatchClasses + 1;
        std::vector<std::pair<double, size_t>> order;
        std::vector<ItemDev> all;
        for (int i = 0; i < n; ++i) {
            pufe_ctx *c = ctxs[i];
            if (pass < split_pass && cls[i] != pass) continue;
            for (const ItemDev &it0 : pass < split_pass ? c->items : (pass == split_pass ? c->items_split : c->items_wide)) {
                ItemDev it = it0;
                it.ctx = i;
                order.push_back({item_cost(it, c->plan.kp.n3), all.size()});
                all.push_back(it);
            }
        }
        std::stable_sort(order.begin(), order.end(),
                         [](const std::pair<double, size_t> &a, const std::pair<double, size_t> &c) { return a.first > c.first; });
        std::vector<ItemDev> &dst = pass < split_pass ? b->items : (pass == split_pass ? b->items_split : b->items_wide);
        for (auto &o : order) dst.push_back(all[o.second]);
        if (pass < split_pass) b->item_off[pass + 1] = (int64_t)b->items.size();
    }
    int cr[kBatchClasses], cf[kBatchClasses], ci[kBatchClasses], cl[kBatchClasses], cn3[kBatchClasses];
    bool all_tuned[kBatchClasses];
    for (int k = 0; k < kBatchClasses; ++k) cr[k] = 16, cf[k] = 1, ci[k] = 0, cl[k] = 1, cn3[k] = 1, all_tuned[k] = true;
    for (int i = 0; i < n; ++i) {
        pufe_ctx *c = ctxs[i];
        const int k = cls[i];
        cr[k] = std::max(cr[k], c->max_rows);
        cf[k] = std::max(cf[k], c->plan.max_nfun);
        ci[k] = std::max(ci[k], c->plan.max_img);
        cl[k] = std::max(cl[k], c->max_item_leaves);
        cn3[k] = std::max(cn3[k], c->plan.kp.n3);
        all_tuned[k] = all_tuned[k] && c->tuned;
        max_rows_split = std::max(max_rows_split, c->max_rows_split);
        max_nfun = std::max(max_nfun, c->plan.max_nfun);
        max_img = std::max(max_img, c->plan.max_img);
        max_leaves_split = std::max(max_leaves_split, c->max_item_leaves_split);
        max_n3 = std::max(max_n3, c->plan.kp.n3);
        b->max_l = std::max(b->max_l, c->plan.max_l);
        b->gen = b->gen || general_variant(c->plan);
        if (!c->items_wide.empty()) b->lds_wide = std::max(b->lds_wide, c->lds_wide);
        for (int64_t e = 0; e < c->plan.nel; ++e) {
            const int T = (c->plan.elems[e].nloc + 15) / 16;
            for (int pp = 0; pp < T * (T + 1) / 2; ++pp)
                b->lists[c->plan.elems[e].color].push_back(make_int4(i, (int)e, pp, 0));
        }
        for (const int2 &r : c->reduce) b->reduce.push_back(make_int4(i, r.x, r.y, 0));
    }
    std::vector<int4> flat;
    b->list_off.assign(1, 0);
    for (auto &l : b->lists) {
        flat.insert(flat.end(), l.begin(), l.end());
        b->list_off.push_back((int64_t)flat.size());
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess || ncu < 1) ncu = 256;
    // a first class runs at its stage length, two work groups per CU.  A
    // second class keeps its length when every member was tuned (the tuner
    // timed that length against its LDS occupancy) or when two work groups
    // still share a CU; otherwise it runs 16-point stages, two per CU.
    for (int k = 0; k < kBatchClasses; ++k) {
        const int qv = kBatchQ[k / 2];
        b->q[k] = qv;
        b->lds_f64[k] = contract_lds_bytes(qv, cr[k], cf[k], ci[k], cl[k], cn3[k]);
        const bool keep = all_tuned[k] && b->lds_f64[k] <= kMaxDynLds;
        if ((k & 1) && qv > 16 && !keep && persistent_blocks_per_cu(b->lds_f64[k]) < 2) {
            b->q[k] = 16;
            b->lds_f64[k] = contract_lds_bytes(16, cr[k], cf[k], ci[k], cl[k], cn3[k]);
        }
        b->grid_f64[k] = ncu * std::max(persistent_blocks_per_cu(b->lds_f64[k]), 1);
    }
    for (int k = 0; k < 2; ++k) {
        b->lds_split[k] = split_lds_bytes(k + 2, max_rows_split, max_nfun, max_img, max_leaves_split, max_n3);
        b->grid_split[k] = ncu * persistent_blocks_per_cu(b->lds_split[k]);
    }
    // the wide items' stage: each problem's own fits, and one wide work group
    // per CU; the largest stage of the problems serves all of them
    {
        int rw = 16, lw = 1;
        for (int i = 0; i < n; ++i)
            if (!ctxs[i]->items_wide.empty()) {
                rw = std::max(rw, ctxs[i]->max_rows_wide);
                lw = std::max(lw, ctxs[i]->max_item_leaves_wide);
            }
        if (!b->items_wide.empty()) b->lds_wide = contract_wide_lds_bytes(rw, max_nfun, max_img, lw, max_n3);
        b->grid_wide = ncu;
    }
    hipStream_t st = nullptr;
    if (b->d_items.upload(b->items, st) != hipSuccess || b->d_items_split.upload(b->items_split, st) != hipSuccess ||
        b->d_items_wide.upload(b->items_wide, st) != hipSuccess ||
        b->d_lists.upload(flat, st) != hipSuccess || b->d_reduce.upload(b->reduce, st) != hipSuccess ||
        b->d_counter.alloc(1) != hipSuccess || b->d_ctxs.alloc(n) != hipSuccess ||
        b->d_ztab.alloc(kMaxKPerLaunch * 27) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return PUFE_ERR_OOM;
    }
    *out = b;
    return PUFE_OK;
}

int pufe_batch_destroy(pufe_batch *b) {
    if (!b) return PUFE_ERR_INVALID_ARG;
    (void)hipSetDevice(b->device);
    delete b;
    return PUFE_OK;
}

int pufe_batch_assemble(pufe_batch *b, const double *const *d_V, const double *kpts, int n_k, int precision,
                        int out_dtype, void *const *d_H, void *const *d_S, void *stream) {
    if (!b) return PUFE_ERR_INVALID_ARG;
    const int n = (int)b->ctxs.size();
    if (!d_V || !d_H || !kpts || n_k < 1 || n_k > kMaxKPerLaunch)
        return bfail(b, PUFE_ERR_INVALID_ARG, "null pointer or n_k outside 1..16");
    if (precision < PUFE_PREC_FP64 || precision > PUFE_PREC_BF16X6 || out_dtype < PUFE_OUT_C128 ||
        out_dtype > PUFE_OUT_F64_GAMMA)
        return bfail(b, PUFE_ERR_INVALID_ARG, "unknown precision or dtype");
    for (int i = 0; i < n; ++i)
        if (!d_V[i] || !d_H[i]) return bfail(b, PUFE_ERR_INVALID_ARG, "null V or H pointer");
    for (int i = 0; i < n; ++i)
        if (b->ctxs[i]->plan_gen != b->gens[i])
            return bfail(b, PUFE_ERR_STATE, "problem " + std::to_string(i) +
                                                " was set up or tuned again after pufe_batch_create; create the batch anew");
    for (int k = 0; k < 3 * n_k; ++k) {
        if (!std::isfinite(kpts[k])) return bfail(b, PUFE_ERR_INVALID_ARG, "non-finite k-point");
        if (out_dtype == PUFE_OUT_F64_GAMMA && std::fmod(kpts[k], 1.0) != 0.0)
            return bfail(b, PUFE_ERR_INVALID_ARG, "real output needs Gamma");
    }
    hipStream_t st = (hipStream_t)stream;
    CHECK_HIP_B(b, hipSetDevice(b->device), "hipSetDevice");
    std::vector<uintptr_t> key;
    key.push_back((uintptr_t)precision);
    key.push_back((uintptr_t)out_dtype);
    key.push_back((uintptr_t)n_k);
    for (int i = 0; i < n; ++i) {
        key.push_back((uintptr_t)d_V[i]);
        key.push_back((uintptr_t)d_H[i]);
        key.push_back((uintptr_t)(d_S ? d_S[i] : nullptr));
    }
    for (int k = 0; k < 3 * n_k; ++k) {
        uint64_t bits;
        std::memcpy(&bits, &kpts[k], sizeof bits);
        key.push_back((uintptr_t)bits);
    }
    if (!b->exec || key != b->key) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        std::vector<CtxDev> cd(n);
        for (int i = 0; i < n; ++i) {
            pufe_ctx *c = b->ctxs[i];
            cd[i].kp = c->plan.kp;
            cd[i].elems = c->d_elems.p;
            cd[i].groups = c->d_groups.p;
            cd[i].img = c->d_img.p;
            cd[i].edof = c->d_edof.p;
            cd[i].leaves = c->d_leaves.p;
            cd[i].V = d_V[i];
            cd[i].partial = c->d_partial.p;
            cd[i].H = d_H[i];
            cd[i].S = d_S ? d_S[i] : nullptr;
            cd[i].nnz = c->plan.nnz;
        }
        CHECK_HIP_B(b, hipMemcpy(b->d_ctxs.p, cd.data(), sizeof(CtxDev) * n, hipMemcpyHostToDevice), "upload tables");
        KPoints kps;
        std::memset(&kps, 0, sizeof kps);
        kps.nk = n_k;
        for (int k = 0; k < n_k; ++k)
            for (int d = 0; d < 3; ++d) kps.kap[k][d] = kpts[3 * k + d];
        CHECK_HIP_B(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture");
        hipError_t e = hipSuccess;
        if (precision == PUFE_PREC_FP64) {
            // one persistent launch per class (the queue counter is reset by each)
            for (int k = 0; k < kBatchClasses && e == hipSuccess; ++k) {
                const int cnt = (int)(b->item_off[k + 1] - b->item_off[k]);
                if (cnt == 0) continue;
                if (b->lds_f64[k] > kMaxDynLds) {
                    e = hipErrorInvalidValue;
                    break;
                }
                e = launch_contract_persistent(b->q[k], b->max_l, b->gen, b->d_ctxs.p, b->d_items.p + b->item_off[k], cnt,
                                               b->d_counter.p, b->grid_f64[k], b->lds_f64[k], b->cap);
            }
            if (e == hipSuccess && !b->items_wide.empty()) {
                if (b->lds_wide > kMaxDynLds) e = hipErrorInvalidValue;
                else
                    e = launch_contract_wide_persistent(b->max_l, b->gen, b->d_ctxs.p, b->d_items_wide.p,
                                                        (int)b->items_wide.size(), b->d_counter.p, b->grid_wide,
                                                        b->lds_wide, b->cap);
            }
        } else {
            const int k = precision == PUFE_PREC_BF16X3 ? 0 : 1;
            if (b->lds_split[k] > kMaxDynLds) e = hipErrorInvalidValue;
            else
                e = launch_split_persistent(k + 2, b->max_l, b->gen, b->d_ctxs.p, b->d_items_split.p, (int)b->items_split.size(), b->d_counter.p,
                                            b->grid_split[k], b->lds_split[k], b->cap);
        }
        if (e == hipSuccess) e = launch_chunk_reduce_batch(b->d_ctxs.p, b->d_reduce.p, (int)b->reduce.size(), b->cap);
        const bool f32 = out_dtype == PUFE_OUT_C64;
        for (int i = 0; i < n && e == hipSuccess; ++i) {
            const int64_t per = (out_dtype == PUFE_OUT_F64_GAMMA ? 1 : 2) * b->ctxs[i]->plan.nnz * n_k;
            e = launch_fill_zero(d_H[i], per, f32, b->cap);
            if (e == hipSuccess && d_S && d_S[i]) e = launch_fill_zero(d_S[i], per, f32, b->cap);
        }
        if (e == hipSuccess) e = launch_phase_table(kps, b->d_ztab.p, b->cap);
        for (size_t col = 0; col + 1 < b->list_off.size() && e == hipSuccess; ++col) {
            const int cnt = (int)(b->list_off[col + 1] - b->list_off[col]);
            e = launch_scatter_batch(b->d_ctxs.p, b->d_lists.p + b->list_off[col], cnt, b->d_ztab.p, n_k, out_dtype,
                                     b->cap);
        }
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->cap, &g);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bfail(b, PUFE_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
        }
        CHECK_HIP_B(b, e2, "end capture");
        b->graph = g;
        CHECK_HIP_B(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate graph");
        b->key = key;
    }
    CHECK_HIP_B(b, hipGraphLaunch(b->exec, st), "graph launch");
    return PUFE_OK;
}

const char *pufe_batch_last_error_message(const pufe_batch *b) { return b ? b->err.c_str() : "no batch"; }

}  // extern "C"
