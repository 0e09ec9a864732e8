// Internal declarations of liblbm: lattice traits, kernel argument blocks and
// the host-side model description.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "lbm.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Velocity sets.  Classes are the shells |e|^2 = 0, 1, 2; every velocity of a
// shell shares one weight and one set of equilibrium coefficients.
// d1v3 and d2v9 are the sets of the section "The Gaussian quadrature" (the
// long d2v9 vectors read as (1,1), (-1,1), (-1,-1), (1,-1)); d3v19 is the
// 19-velocity set whose weights solve the same moment conditions in D = 3.
// ---------------------------------------------------------------------------
struct D1Q3 {
    static constexpr int D = 1, Q = 3;
    static constexpr int e[Q][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}};
    static constexpr int cls[Q] = {0, 1, 1};
    static constexpr int opp[Q] = {0, 2, 1};
};

struct D2Q9 {
    static constexpr int D = 2, Q = 9;
    static constexpr int e[Q][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                                    {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    static constexpr int cls[Q] = {0, 1, 1, 1, 1, 2, 2, 2, 2};
    static constexpr int opp[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
};

struct D3Q19 {
    static constexpr int D = 3, Q = 19;
    static constexpr int e[Q][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                                    {0, 0, 1},  {0, 0, -1}, {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
                                    {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    static constexpr int cls[Q] = {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};
    static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
};

// ---------------------------------------------------------------------------
// Host model: per-class equilibrium coefficients in float64.
// f_eq,a = n w_k S_a with S_a - 1 = eu (l1 + c3 u^2 + k4 eu^2) + q eu^2 + s u^2.
// ---------------------------------------------------------------------------
struct ClassCoef {
    double w, l1, q, s, c3, k4;
};

struct Model {
    int D = 0, Q = 0, ncls = 0;
    ClassCoef cls[3] = {};
    double J2 = 0, J4 = 0, d2sq = 0, d4sq = 0;
};

// Validates cfg and fills the model.  Returns LBM_OK or an error with text in err.
lbm_status build_model(const lbm_config *cfg, Model *m, std::string *err);

// ---------------------------------------------------------------------------
// Kernel argument block (passed by value: it lives in the kernel-argument
// segment, read through scalar loads, i.e. the constant path of the CU).
// ---------------------------------------------------------------------------
template <typename T>
struct Coef {
    T w[3], l1[3], q[3], s[3], c3[3], k4[3];
    T omega, rho_ref;
};

struct Box {
    int nx, ny, nz;
    int bbx, bby, bbz;  // 1 = halfway bounce-back on that axis, 0 = periodic
    int64_t plane;      // distance between population planes (elements): cells plus a pad
    int64_t cells;      // nx ny nz: distance between the components of a field (n, u)
};

// Constant body force (force density per cell and step, lattice units).
template <typename T>
struct Force {
    T F[3];
};

// Per-cell link mask of a box with solid cells: bit a set when the link
// x -> x + e_a ends in a solid cell (links that leave the box through a wall
// face are handled by the wall flags), bit 31 set when the cell is solid.
constexpr uint32_t kSolidBit = 0x80000000u;

}  // namespace lbm
