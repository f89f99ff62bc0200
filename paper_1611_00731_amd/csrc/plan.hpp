// Host planner: from the problem statement to the tables the kernels read.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pufe.h"
#include "tables.hpp"

namespace pufe {

struct Problem {
    double lat[9];
    int mesh[3];
    int p;
    std::vector<double> pos;  // n_atoms x 3
    std::vector<int> species;
    std::vector<pufe_enrichment> enr;            // radial pointers cleared
    std::vector<std::vector<double>> radial;     // samples of tabulated radials, per descriptor
    pufe_quad quad;
    std::vector<pufe_projector> proj;   // separable nonlocal term (may be empty)
    int enr_phase = PUFE_ENR_PERIODIC;  // f(R) of eq. Psi
};

struct Plan {
    // cell
    double lat[9], inv[9], vol;
    int64_t nel, nv;
    int nfs, nfe;
    // enriched functions of each vertex: (atom, desc, m)
    std::vector<int64_t> vf_off;
    std::vector<int32_t> vf;  // 3 per function
    std::vector<int64_t> dof_off;
    // block-sparse layout keyed by vertex
    std::vector<int64_t> brow_ptr, bval_off;
    std::vector<int32_t> bcol, brow;
    int64_t nnz = 0;
    // elements
    std::vector<ElemDev> elems;
    std::vector<GroupDev> groups;
    std::vector<double> img;        // image centres at the planned positions, 3 per image
    std::vector<double> img_cur;    // image centres at the current positions
    std::vector<int32_t> edof;      // packed enriched local functions
    // Bloch-periodic enrichment: every (atom, descriptor) group of an element
    // is followed by a copy that evaluates the imaginary part (image weights
    // sin instead of cos), and every enriched local function by its
    // imaginary-part partner in the same PU corner
    bool bloch = false;
    std::vector<int32_t> img_nk;    // per image entry: lattice shift n (3), then 0 (cos weight) or 1 (sin)
    std::vector<int32_t> bpart;     // per enriched entry: its partner's entry index (-1: an imaginary part)
    std::vector<int32_t> color_elems;
    std::vector<int32_t> color_off; // n_colors + 1
    std::vector<int2> scat;         // (element, upper tile pair), colour by colour
    std::vector<int64_t> scat_off;  // n_colors + 1
    int max_nloc = 0, max_nfun = 0, max_ngrp = 0;
    int max_l = 0;                  // largest angular momentum of any descriptor
    int max_img = 0;                // most image centres of one element's groups
    // tabulated radials: 4 power coefficients per interval, per descriptor
    std::vector<double> spl;
    std::vector<int32_t> spl_off;   // per descriptor (-1 analytic)
    KParams kp;
    // separable nonlocal term: projector functions J (atom, descriptor, m)
    // with their weights, the projector-image groups of every element, and
    // for every DOF the (element, local function) pairs that carry it
    int n_pfun = 0;
    std::vector<double> pfun_h;
    std::vector<PGroupDev> pgroups;
    std::vector<int64_t> dof_el_off;  // n_dof + 1
    std::vector<int2> dof_el;         // (element, local function)
    int max_ncol = 0, max_npg = 0;
    std::vector<int32_t> nl_blocks;   // BSR blocks coupled through a projector image
};

// Image lists keep every image within rc + this margin of an element, so the
// enrichment centres may move by up to the margin without replanning.
constexpr double kImageMargin = 0.25;

// Validate and plan; returns PUFE_OK or an error code with a message.
int build_plan(const Problem &pr, Plan &pl, std::string &err);

}  // namespace pufe
