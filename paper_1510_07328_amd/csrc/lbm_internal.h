// Internal declarations of liblbm: lattice traits, kernel argument blocks and
// the host-side model description.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "lbm.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Velocity sets.  Classes are the shells |e|^2 = const; every velocity of a
// shell shares one weight and one set of equilibrium coefficients.  R is the
// longest link along x (cells), NC the number of classes, O4 marks a set exact
// to degree 9 that carries the fourth-order terms, MAXB the largest workgroup
// its kernels are compiled for (the register budget of a thread).
// d1v3 and d2v9 are the sets of the section "The Gaussian quadrature" (the
// long d2v9 vectors read as (1,1), (-1,1), (-1,-1), (1,-1)); d3v19 is the
// 19-velocity set whose weights solve the same moment conditions in D = 3;
// d2v41 (shells |e|^2 = 0, 1, 2, 4, 8, 9, 10, 13, 16) is a set whose weights
// solve them through degree 9, for the fourth-order expansion.
// ---------------------------------------------------------------------------
constexpr int kMaxClasses = 9;

struct D1Q3 {
    static constexpr int D = 1, Q = 3, R = 1, NC = 2, MAXB = 1024;
    static constexpr bool O4 = false;
    static constexpr int e[Q][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}};
    static constexpr int cls[Q] = {0, 1, 1};
    static constexpr int opp[Q] = {0, 2, 1};
};

struct D2Q9 {
    static constexpr int D = 2, Q = 9, R = 1, NC = 3, MAXB = 1024;
    static constexpr bool O4 = false;
    static constexpr int e[Q][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},   {-1, 0, 0}, {0, -1, 0},
                                    {1, 1, 0},  {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
    static constexpr int cls[Q] = {0, 1, 1, 1, 1, 2, 2, 2, 2};
    static constexpr int opp[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
};

struct D3Q19 {
    static constexpr int D = 3, Q = 19, R = 1, NC = 3, MAXB = 1024;
    static constexpr bool O4 = false;
    static constexpr int e[Q][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                                    {0, 0, 1},  {0, 0, -1}, {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
                                    {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    static constexpr int cls[Q] = {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};
    static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
};

// Velocities in (v, -v) pairs, shell by shell.
struct D2Q41 {
    static constexpr int D = 2, Q = 41, R = 4, NC = 9, MAXB = 512;
    static constexpr bool O4 = true;
    static constexpr int e[Q][3] = {
        {0, 0, 0},   {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},  {1, 1, 0},  {-1, -1, 0}, {-1, 1, 0},
        {1, -1, 0},  {2, 0, 0},   {-2, 0, 0}, {0, 2, 0},   {0, -2, 0},  {2, 2, 0},  {-2, -2, 0}, {-2, 2, 0},
        {2, -2, 0},  {3, 0, 0},   {-3, 0, 0}, {0, 3, 0},   {0, -3, 0},  {3, 1, 0},  {-3, -1, 0}, {1, 3, 0},
        {-1, -3, 0}, {-1, 3, 0},  {1, -3, 0}, {-3, 1, 0},  {3, -1, 0},  {3, 2, 0},  {-3, -2, 0}, {2, 3, 0},
        {-2, -3, 0}, {-2, 3, 0},  {2, -3, 0}, {-3, 2, 0},  {3, -2, 0},  {4, 0, 0},  {-4, 0, 0},  {0, 4, 0},
        {0, -4, 0}};
    static constexpr int cls[Q] = {0, 1, 1, 1, 1, 2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4, 5, 5, 5, 5,
                                   6, 6, 6, 6, 6, 6, 6, 6, 7, 7, 7, 7, 7, 7, 7, 7, 8, 8, 8, 8};
    static constexpr int opp[Q] = {0,  2,  1,  4,  3,  6,  5,  8,  7,  10, 9,  12, 11, 14,
                                   13, 16, 15, 18, 17, 20, 19, 22, 21, 24, 23, 26, 25, 28,
                                   27, 30, 29, 32, 31, 34, 33, 36, 35, 38, 37, 40, 39};
    static constexpr int shell[NC] = {0, 1, 2, 4, 8, 9, 10, 13, 16};  // |e|^2 of each class
};

// ---------------------------------------------------------------------------
// Host model: per-class equilibrium coefficients in float64.
// f_eq,a = n w_k S_a with
//   S_a - 1 = eu (l1 + c3 u^2 + k4 eu^2) + q eu^2 + s u^2
//           + p4 eu^4 + r4 eu^2 u^2 + t4 u^4          (fourth order, d2v41 only).
// ---------------------------------------------------------------------------
struct ClassCoef {
    double w, l1, q, s, c3, k4, p4, r4, t4;
};

struct Model {
    int D = 0, Q = 0, ncls = 0;
    int lattice = 0;  // lbm_lattice
    ClassCoef cls[kMaxClasses] = {};
    double scale = 0;  // c_0 / sqrt(3 I_4 / I_2) of the set (1 except d2v41)
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
    T w[kMaxClasses], l1[kMaxClasses], q[kMaxClasses], s[kMaxClasses], c3[kMaxClasses], k4[kMaxClasses];
    T p4[kMaxClasses], r4[kMaxClasses], t4[kMaxClasses];  // fourth order (d2v41)
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
