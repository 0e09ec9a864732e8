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
    int local = 0;   // LBM_W_FD_LOCAL: weights and coefficients per cell from its density
    double r0 = 0;   // theta / mu at the reference density
};

// Validates cfg and fills the model.  Returns LBM_OK or an error with text in err.
lbm_status build_model(const lbm_config *cfg, Model *m, std::string *err);

// ---------------------------------------------------------------------------
// Kernel argument block (passed by value: it lives in the kernel-argument
// segment, read through scalar loads, i.e. the constant path of the CU).
// ---------------------------------------------------------------------------
// Per-cell weights (LBM_W_FD_LOCAL): what a cell needs to find J_2, J_4 from
// its density n.  x = n / rho_ref = 1 + dm; mu / mu_ref solves
// (mu/mu_ref)^(D/2) [1 + b_0 r2 (mu_ref/mu)^2] = x rhs, rhs = 1 + b_0 r2;
// t = r2 (mu_ref/mu)^2 = r2 + dt; B_N = Br_N + b_N dt (Br_N at the reference);
// J_4 = J4z B_2^2 / (B_1 B_3) and J_2 = J2r + dJ2 with the difference formed
// without cancellation, dJ2 = J2z dt (P1 + P2 dt) / (B_0 B_2 Br_0 Br_2).
template <typename T>
struct LocalW {
    T r2;         // (theta / mu_ref)^2
    T b[4];       // (pi^2/6) nu (nu - 1), nu = N + D/2
    T J2z, J4z;   // zero-temperature J_2, J_4
    T rhs;        // 1 + b_0 r2
    T inv_rho;    // 1 / rho_ref
    T Br[4];      // B_N at the reference state
    T J2r;        // J_2 at the reference state
    T P1, P2;     // numerator of J_2 - J2r, divided by dt J2z
    T inv_br02;   // 1 / (Br_0 Br_2)
};

template <typename T>
struct Coef {
    T w[3], l1[3], q[3], s[3], c3[3], k4[3];
    T omega, rho_ref;
    LocalW<T> loc;  // used by the per-cell weight kernels only
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
