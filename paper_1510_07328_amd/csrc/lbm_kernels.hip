// HIP kernels of the lattice BGK step for gfx950.
//
// One fused kernel per time step (lattice BGK equation and the moment update
// that follows it, section "The Gaussian quadrature"):
//   moments dn = sum_a g_a, j = sum_a g_a e_a, n = rho_ref + dn, u0 = j / n,
//   equilibrium g_eq,a = w_a [dn + n (S_a - 1)] from the per-class polynomial,
//   relax   g_a <- g_a + (g_eq,a - g_a) / tau,
//   stream  to x + e_a (periodic wrap, or halfway bounce-back at walls).
// Populations are deviations g = f - w rho_ref, so f_eq - w rho_ref is formed
// without the 1 - 1 cancellation and small drifts survive in float32.
//
// The weights are rounded to the storage precision so that, as real numbers,
// sum_a w_a = 1 and sum_a w_a e_ax^2 = c_s^2 hold exactly for the rounded values
// whenever c_s^2 = J_2 / 3 is representable (it is 1/2 on d2v9 at theta = 0):
// w_short = fl(J2/9), w_long = (c_s^2 - 2 w_short) / 4, w_rest = 1 - 4 w_short
// - 4 w_long, each exact.  The equilibrium's pressure, and with it the sound
// speed, then carries no rounding of the weights; rounding each weight on its
// own shifts c_s^2 by about 3e-8 in float32, which accumulates as phase error of
// the acoustic waves (1e-5 relative after 1e4 steps on the 2048^2 field).
//
// Layout: structure of arrays g[a][z][y][x], x fastest, the population planes
// Box::plane elements apart (the cell count plus a pad: planes a power of two
// apart would put the same address bits, and so the same HBM channels, under
// all 18 streams of a step at once).  One workgroup owns one
// (y, z) row and its threads stride over x, so every wavefront load and store
// of a population is a contiguous run of 64 lanes (256 B in float32), x wrap
// stays inside the workgroup, and no cache line is shared between workgroups
// on different XCDs (streaming is a permutation: each value is written by
// exactly one cell and read by exactly one cell).
//
// Two streaming schemes, both "collide then stream", so both hold the
// post-streaming populations after every step and agree bit for bit:
//   push  reads the cell's own slots of lattice A, writes x + e_a of lattice B
//         (two lattices in HBM);
//   AA    in place on one lattice: even steps read and write the cell's own
//         slots (writing a to the slot of -a), odd steps read the slots of -a
//         at x - e_a and write slot a at x + e_a.  Each location is read and
//         written by the same cell only, so no two cells race.
#include <hip/hip_runtime.h>

#include "lbm_collide.h"
#include "lbm_internal.h"

namespace lbm {

// Row offsets of the cells x + sign e_a for every a, resolved once per row
// (block-uniform, so they live in scalar registers).  rowbb[a] marks a link
// that leaves the box through a bounce-back face in y or z.
template <class L>
__device__ __forceinline__ void row_links(const Box &b, int y, int z, int sign, int64_t (&rowoff)[L::Q],
                                          bool (&rowbb)[L::Q]) {
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        int ys = y + sign * L::e[q][1], zs = z + sign * L::e[q][2];
        bool bb = false;
        if (ys < 0 || ys >= b.ny) {
            if (b.bby) bb = true;
            else ys = ys < 0 ? ys + b.ny : ys - b.ny;
        }
        if (zs < 0 || zs >= b.nz) {
            if (b.bbz) bb = true;
            else zs = zs < 0 ? zs + b.nz : zs - b.nz;
        }
        rowoff[q] = bb ? int64_t(0) : ((int64_t)zs * b.ny + ys) * b.nx;
        rowbb[q] = bb;
    }
}

// Bit a of a cell's link mask (the link x -> x + e_a ends in a solid cell).
// Sets with 32 links or more carry no mask; the test is then false, and the
// shift, which would be undefined for a 32-bit mask, is never formed (a is a
// compile-time constant in the unrolled loops).
__device__ __forceinline__ bool link_bit(uint32_t m, int a) { return a < 32 && ((m >> a) & 1u); }

// x + dx with periodic wrap; sets bb when the link leaves through a wall.
// Written with selects only (no branches): the wrap or the wall concerns the
// two ends of a row, and the callers pick the slot address with a select too,
// so each of the Q loads and stores is one unconditional memory instruction.
__device__ __forceinline__ int link_x(const Box &b, int x, int dx, bool &bb) {
    if (dx == 0) return x;
    const int xs = x + dx;
    const bool lo = xs < 0, hi = xs >= b.nx;
    bb = bb | ((lo | hi) & (b.bbx != 0));
    return lo ? xs + b.nx : (hi ? xs - b.nx : xs);
}

// Slot addresses.  A lattice below 4 GiB is addressed with 32-bit byte
// offsets from its base: a block-uniform offset then takes one scalar register
// and each load or store is base + 32-bit lane offset, so the 2Q per-row
// offsets of the odd AA and push steps stay in scalar registers (on d3v19 the
// 64-bit form of those offsets spilled).  Larger lattices take 64-bit element
// offsets (WIDE).
template <typename T, bool WIDE>
struct Slot;

template <typename T>
struct Slot<T, false> {
    using off = uint32_t;
    static __device__ __forceinline__ off of(int64_t elem) { return uint32_t(elem) * uint32_t(sizeof(T)); }
    static __device__ __forceinline__ T &at(T *p, off o) { return *reinterpret_cast<T *>(reinterpret_cast<char *>(p) + o); }
    static __device__ __forceinline__ T at(const T *p, off o) {
        return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + o);
    }
};

template <typename T>
struct Slot<T, true> {
    using off = int64_t;
    static __device__ __forceinline__ off of(int64_t elem) { return elem; }
    static __device__ __forceinline__ T &at(T *p, off o) { return p[o]; }
    static __device__ __forceinline__ T at(const T *p, off o) { return p[o]; }
};

// Populations of the cell x that the odd AA step collides: slot -a at x - e_a,
// or, where that link crosses a wall face or ends in a solid cell (bit -a of
// the link mask m), the cell's own slot a, written there by the reflection.
template <class L, typename T>
__device__ __forceinline__ void load_natural(const T *__restrict__ lat, const Box &b, int x, int64_t own_row,
                                             const int64_t (&inoff)[L::Q], const bool (&inbb)[L::Q], bool odd,
                                             uint32_t m, T (&g)[L::Q]) {
    if (!odd) {
#pragma unroll
        for (int q = 0; q < L::Q; ++q) g[q] = lat[q * b.plane + own_row + x];
    } else {
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            bool bb = inbb[q];
            const int xs = link_x(b, x, -L::e[q][0], bb);
            bb = bb || link_bit(m, L::opp[q]);
            g[q] = lat[bb ? q * b.plane + own_row + x : L::opp[q] * b.plane + inoff[q] + xs];
        }
    }
}

// Block-uniform slot offsets of a row's interior cells (x - R and x + R in the
// row): in[q] + x is where the odd AA step reads population q (slot -q at
// x - e_q, or the cell's own slot q when the link crosses a wall face in y or
// z), out[q] + x where the push and odd AA steps write it (slot q at x + e_q,
// or the own slot -q at a wall).
template <class L, typename S>
__device__ __forceinline__ void interior_slots(const Box &b, typename S::off (&in)[L::Q],
                                               typename S::off (&out)[L::Q]) {
    const int row = blockIdx.x;
    const int y = row % b.ny, z = row / b.ny;
    const int64_t own_row = (int64_t)row * b.nx;
    int64_t off[L::Q];
    bool bb[L::Q];
    row_links<L>(b, y, z, -1, off, bb);
#pragma unroll
    for (int q = 0; q < L::Q; ++q)
        in[q] = S::of(bb[q] ? q * b.plane + own_row : L::opp[q] * b.plane + off[q] - L::e[q][0]);
    row_links<L>(b, y, z, +1, off, bb);
#pragma unroll
    for (int q = 0; q < L::Q; ++q)
        out[q] = S::of(bb[q] ? L::opp[q] * b.plane + own_row : q * b.plane + off[q] + L::e[q][0]);
}

// True when the link from the workgroup's row to the row y + sign e_qy,
// z + sign e_qz leaves through a bounce-back face in y or z.
template <class L>
__device__ __forceinline__ bool wall_yz(const Box &b, int q, int sign) {
    const int row = blockIdx.x;
    const int ys = row % b.ny + sign * L::e[q][1], zs = row / b.ny + sign * L::e[q][2];
    return (b.bby && (ys < 0 || ys >= b.ny)) || (b.bbz && (zs < 0 || zs >= b.nz));
}

// The cells at the two ends of a row (the L::R cells at each end, where a link
// can wrap round the row or leave through a wall face in x): the interior
// offsets in/out plus, per lane, the wrap (+-nx) or the reflection into the
// cell's own slot.  Run by the first 2 L::R threads of the workgroup after its
// interior loop; no other cell reads or writes their slots.  `odd` selects the odd AA
// gather (else the cell's own slots of src); the store is the push / odd AA
// store into dst.
template <class L, typename T, class S, bool O3, bool POROUS, bool LOCAL = false>
__device__ __forceinline__ void row_ends(const T *src, T *dst, const uint32_t *__restrict__ lm, const Box &b,
                                         bool odd, const typename S::off (&in)[L::Q],
                                         const typename S::off (&out)[L::Q], const Coef<T> &c, const T *F) {
    using off = typename S::off;
    const int ends = b.nx < 2 * L::R ? b.nx : 2 * L::R;
    const int t = threadIdx.x;
    if (t >= ends) return;
    const int x = b.nx <= 2 * L::R ? t : (t < L::R ? t : b.nx - 2 * L::R + t);
    const int64_t own_row = (int64_t)blockIdx.x * b.nx;
    const uint32_t m = POROUS ? lm[own_row + x] : 0u;
    if (m & kSolidBit) return;
    const off own = S::of(own_row + x), pl = S::of(b.plane), ox = S::of(x), onx = S::of(b.nx);
    T g[L::Q];
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        if (!odd) {
            g[q] = S::at(src, q * pl + own);
            continue;
        }
        const int xs = x - L::e[q][0];
        const bool lo = xs < 0, hi = xs >= b.nx;
        const bool bb = link_bit(m, L::opp[q]) || ((lo || hi) && b.bbx);
        const off wrap = wall_yz<L>(b, q, -1) ? off(0) : (lo ? onx : (hi ? off(0) - onx : off(0)));
        g[q] = S::at(src, bb ? q * pl + own : in[q] + ox + wrap);
    }
    collide<L, T, O3, POROUS, LOCAL>(g, c, F);
#pragma unroll
    for (int q = 0; q < L::Q; ++q) {
        const int xt = x + L::e[q][0];
        const bool lo = xt < 0, hi = xt >= b.nx;
        const bool bb = link_bit(m, q) || ((lo || hi) && b.bbx);
        const off wrap = wall_yz<L>(b, q, +1) ? off(0) : (lo ? onx : (hi ? off(0) - onx : off(0)));
        S::at(dst, bb ? L::opp[q] * pl + own : out[q] + ox + wrap) = g[q];
    }
}

// ---------------------------------------------------------------------------
// push step: collide at the cell, stream into the other lattice
// ---------------------------------------------------------------------------
template <class L, typename T, bool O3, bool W, bool LOCAL>
__global__ void __launch_bounds__(L::MAXB) k_push(const T *__restrict__ src, T *__restrict__ dst, Box b, Coef<T> c) {
    using S = Slot<T, W>;
    typename S::off in[L::Q], out[L::Q];
    interior_slots<L, S>(b, in, out);
    const typename S::off own = S::of((int64_t)blockIdx.x * b.nx), pl = S::of(b.plane);
    for (int x = threadIdx.x; x < b.nx; x += blockDim.x) {
        if (x < L::R || x >= b.nx - L::R) continue;
        const typename S::off ox = S::of(x);
        T g[L::Q];
#pragma unroll
        for (int q = 0; q < L::Q; ++q) g[q] = S::at(src, q * pl + own + ox);
        collide<L, T, O3, false, LOCAL>(g, c);
#pragma unroll
        for (int q = 0; q < L::Q; ++q) S::at(dst, out[q] + ox) = g[q];
    }
    row_ends<L, T, S, O3, false, LOCAL>(src, dst, nullptr, b, false, in, out, c, nullptr);
}

// ---------------------------------------------------------------------------
// AA steps, in place
// ---------------------------------------------------------------------------
template <class L, typename T, bool O3, bool W, bool LOCAL>
__global__ void __launch_bounds__(L::MAXB) k_aa_even(T *__restrict__ lat, Box b, Coef<T> c) {
    using S = Slot<T, W>;
    const typename S::off own = S::of((int64_t)blockIdx.x * b.nx), pl = S::of(b.plane);
    for (int x = threadIdx.x; x < b.nx; x += blockDim.x) {
        const typename S::off o = own + S::of(x);
        T g[L::Q];
#pragma unroll
        for (int q = 0; q < L::Q; ++q) g[q] = S::at(lat, q * pl + o);
        collide<L, T, O3, false, LOCAL>(g, c);
#pragma unroll
        for (int q = 0; q < L::Q; ++q) S::at(lat, L::opp[q] * pl + o) = g[q];
    }
}

template <class L, typename T, bool O3, bool W, bool LOCAL>
__global__ void __launch_bounds__(L::MAXB) k_aa_odd(T *__restrict__ lat, Box b, Coef<T> c) {
    using S = Slot<T, W>;
    typename S::off in[L::Q], out[L::Q];
    interior_slots<L, S>(b, in, out);
    for (int x = threadIdx.x; x < b.nx; x += blockDim.x) {
        if (x < L::R || x >= b.nx - L::R) continue;
        const typename S::off ox = S::of(x);
        T g[L::Q];
#pragma unroll
        for (int q = 0; q < L::Q; ++q) g[q] = S::at(lat, in[q] + ox);
        collide<L, T, O3, false, LOCAL>(g, c);
#pragma unroll
        for (int q = 0; q < L::Q; ++q) S::at(lat, out[q] + ox) = g[q];
    }
    row_ends<L, T, S, O3, false, LOCAL>(lat, lat, nullptr, b, true, in, out, c, nullptr);
}

// ---------------------------------------------------------------------------
// Porous-medium steps: solid cells (halfway bounce-back at every link that
// ends in one) and a constant body force (exact difference of equilibria in
// collide()).  Same patterns as above; a solid cell takes no part, and a link
// is reflected when its wall flag or its bit of the cell's link mask is set.
// ---------------------------------------------------------------------------
template <class L, typename T, bool O3, bool W>
__global__ void __launch_bounds__(1024) k_push_p(const T *__restrict__ src, T *__restrict__ dst,
                                                 const uint32_t *__restrict__ lm, Box b, Coef<T> c, Force<T> F) {
    using S = Slot<T, W>;
    typename S::off in[L::Q], out[L::Q];
    interior_slots<L, S>(b, in, out);
    const int64_t own_row = (int64_t)blockIdx.x * b.nx;
    const typename S::off own = S::of(own_row), pl = S::of(b.plane);
    for (int x = threadIdx.x; x < b.nx; x += blockDim.x) {
        if (x < L::R || x >= b.nx - L::R) continue;
        const uint32_t m = lm[own_row + x];
        if (m & kSolidBit) continue;
        const typename S::off ox = S::of(x);
        T g[L::Q];
#pragma unroll
        for (int q = 0; q < L::Q; ++q) g[q] = S::at(src, q * pl + own + ox);
        collide<L, T, O3, true>(g, c, F.F);
#pragma unroll
        for (int q = 0; q < L::Q; ++q)
            S::at(dst, link_bit(m, q) ? L::opp[q] * pl + own + ox : out[q] + ox) = g[q];
    }
    row_ends<L, T, S, O3, true>(src, dst, lm, b, false, in, out, c, F.F);
}

template <class L, typename T, bool O3, bool W>
__global__ void __launch_bounds__(1024) k_aa_even_p(T *__restrict__ lat, const uint32_t *__restrict__ lm, Box b,
                                                    Coef<T> c, Force<T> F) {
    using S = Slot<T, W>;
    const int64_t own_row = (int64_t)blockIdx.x * b.nx;
    const typename S::off own = S::of(own_row), pl = S::of(b.plane);
    for (int x = threadIdx.x; x < b.nx; x += blockDim.x) {
        if (lm[own_row + x] & kSolidBit) continue;
        const typename S::off o = own + S::of(x);
        T g[L::Q];
#pragma unroll
        for (int q = 0; q < L::Q; ++q) g[q] = S::at(lat, q * pl + o);
        collide<L, T, O3, true>(g, c, F.F);
#pragma unroll
        for (int q = 0; q < L::Q; ++q) S::at(lat, L::opp[q] * pl + o) = g[q];
    }
}

template <class L, typename T, bool O3, bool W>
__global__ void __launch_bounds__(1024) k_aa_odd_p(T *__restrict__ lat, const uint32_t *__restrict__ lm, Box b,
                                                   Coef<T> c, Force<T> F) {
    using S = Slot<T, W>;
    typename S::off in[L::Q], out[L::Q];
    interior_slots<L, S>(b, in, out);
    const int64_t own_row = (int64_t)blockIdx.x * b.nx;
    const typename S::off own = S::of(own_row), pl = S::of(b.plane);
    for (int x = threadIdx.x; x < b.nx; x += blockDim.x) {
        if (x < L::R || x >= b.nx - L::R) continue;
        const uint32_t m = lm[own_row + x];
        if (m & kSolidBit) continue;
        const typename S::off ox = S::of(x);
        T g[L::Q];
#pragma unroll
        for (int q = 0; q < L::Q; ++q)  // the cell x - e_q solid: the own slot q, written by the reflection
            g[q] = S::at(lat, link_bit(m, L::opp[q]) ? q * pl + own + ox : in[q] + ox);
        collide<L, T, O3, true>(g, c, F.F);
#pragma unroll
        for (int q = 0; q < L::Q; ++q)
            S::at(lat, link_bit(m, q) ? L::opp[q] * pl + own + ox : out[q] + ox) = g[q];
    }
    row_ends<L, T, S, O3, true>(lat, lat, lm, b, true, in, out, c, F.F);
}

// Link mask from a solid mask (bytes, nonzero = solid).
template <class L>
__global__ void __launch_bounds__(1024) k_link_mask(const unsigned char *__restrict__ solid,
                                                    uint32_t *__restrict__ lm, Box b) {
    const int row = blockIdx.x;
    const int y = row % b.ny, z = row / b.ny;
    int64_t outoff[L::Q];
    bool outbb[L::Q];
    row_links<L>(b, y, z, +1, outoff, outbb);
    const int64_t own_row = (int64_t)row * b.nx;
    for (int x = threadIdx.x; x < b.nx; x += blockDim.x) {
        uint32_t m = solid[own_row + x] ? kSolidBit : 0u;
#pragma unroll
        for (int q = 1; q < L::Q; ++q) {
            bool bb = outbb[q];
            const int xt = link_x(b, x, L::e[q][0], bb);
            if (!bb && solid[outoff[q] + xt]) m |= 1u << q;
        }
        lm[own_row + x] = m;
    }
}

// ---------------------------------------------------------------------------
// initial condition: g = f_eq(n0, u0) - w rho_ref, formed in float64
// ---------------------------------------------------------------------------
template <class L, typename T, bool LOCAL>
__global__ void __launch_bounds__(L::MAXB) k_init(T *__restrict__ lat, const double *__restrict__ n0,
                                               const double *__restrict__ u0, Box b, Coef<double> c, int order3) {
    const int row = blockIdx.x;
    const int64_t own_row = (int64_t)row * b.nx;
    for (int x = threadIdx.x; x < b.nx; x += blockDim.x) {
        const int64_t cell = own_row + x;
        const double n = n0[cell];
        double u[3] = {0.0, 0.0, 0.0}, u2 = 0.0;
#pragma unroll
        for (int d = 0; d < L::D; ++d) {
            u[d] = u0[d * b.cells + cell];
            u2 += u[d] * u[d];
        }
        Classes<double, L::NC> K;
        double dw[L::NC] = {};
        if constexpr (LOCAL) {
            double dJ2;
            ClassSet<double> loc;
            local_classes<L, double>(c.loc, n, n - c.rho_ref, order3 != 0, loc, dJ2);
            for (int k = 0; k < L::NC; ++k) {
                dw[k] = dJ2 * WeightSlope<L>::v[k];
                K.w[k] = c.w[k] + dw[k];
                K.l1[k] = loc.l1[k];
                K.q[k] = loc.q[k];
                K.s[k] = loc.s[k];
                K.c3[k] = loc.c3[k];
                K.k4[k] = loc.k4[k];
                K.p4[k] = K.r4[k] = K.t4[k] = 0.0;
            }
        } else {
            for (int k = 0; k < L::NC; ++k) {
                K.w[k] = c.w[k];
                K.l1[k] = c.l1[k];
                K.q[k] = c.q[k];
                K.s[k] = c.s[k];
                K.c3[k] = c.c3[k];
                K.k4[k] = c.k4[k];
                K.p4[k] = c.p4[k];
                K.r4[k] = c.r4[k];
                K.t4[k] = c.t4[k];
            }
        }
        const double dn = n - c.rho_ref;
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            const int k = L::cls[q];
            double eu = 0.0;
#pragma unroll
            for (int d = 0; d < L::D; ++d) eu += L::e[q][d] * u[d];
            const double sm1 = eu * (K.l1[k] + K.c3[k] * u2 + K.k4[k] * eu * eu) + K.q[k] * eu * eu + K.s[k] * u2 +
                               eu * eu * (K.p4[k] * eu * eu + K.r4[k] * u2) + K.t4[k] * u2 * u2;
            // deviation from the reference weight: w_a(n) n S_a - w_a,ref rho_ref
            lat[q * b.plane + cell] = T(K.w[k] * (dn + n * sm1) + dw[k] * c.rho_ref);
        }
    }
}

// ---------------------------------------------------------------------------
// moments and totals.  `odd` selects the AA read pattern after an odd number
// of steps (populations sit in the slots of -a, still to be streamed).
// ---------------------------------------------------------------------------
// With a link mask (lm not null) solid cells report n = 0, u = 0; with a body
// force F the velocity is the forced scheme's (j + F/2) / n.
// Rows row0 .. row0 + gridDim.x - 1; the output holds those rows from its start,
// n_out[r nx + x] and u_out[d ostride + r nx + x] with r = row - row0 (the whole
// box: row0 = 0, ostride = cells).
template <class L, typename T>
__global__ void __launch_bounds__(L::MAXB) k_moments(const T *__restrict__ lat, double *__restrict__ n_out,
                                                  double *__restrict__ u_out, Box b, double rho_ref, int odd,
                                                  const uint32_t *__restrict__ lm, Force<double> F, int row0,
                                                  int64_t ostride) {
    const int row = row0 + blockIdx.x;
    const int y = row % b.ny, z = row / b.ny;
    int64_t inoff[L::Q];
    bool inbb[L::Q];
    row_links<L>(b, y, z, -1, inoff, inbb);
    const int64_t own_row = (int64_t)row * b.nx;
    const int64_t out_row = (int64_t)blockIdx.x * b.nx;
    for (int x = threadIdx.x; x < b.nx; x += blockDim.x) {
        const uint32_t m = lm ? lm[own_row + x] : 0u;
        if (m & kSolidBit) {
            n_out[out_row + x] = 0.0;
#pragma unroll
            for (int d = 0; d < L::D; ++d) u_out[d * ostride + out_row + x] = 0.0;
            continue;
        }
        T g[L::Q];
        load_natural<L, T>(lat, b, x, own_row, inoff, inbb, odd != 0, m, g);
        double dn = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            dn += double(g[q]);
#pragma unroll
            for (int d = 0; d < L::D; ++d) j[d] += L::e[q][d] * double(g[q]);
        }
        const double n = rho_ref + dn;
        n_out[out_row + x] = n;
#pragma unroll
        for (int d = 0; d < L::D; ++d) u_out[d * ostride + out_row + x] = (j[d] + 0.5 * F.F[d]) / n;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Per-row partial totals part[row][0..4] = {sum n, sum n u0_x, sum n u0_y,
// sum n u0_z, number of cells whose density is not finite and positive}.
// Solid cells (lm not null) are left out.
template <class L, typename T>
__global__ void __launch_bounds__(L::MAXB) k_totals_rows(const T *__restrict__ lat, double *__restrict__ part, Box b,
                                                      double rho_ref, int odd, const uint32_t *__restrict__ lm) {
    const int row = blockIdx.x;
    const int y = row % b.ny, z = row / b.ny;
    int64_t inoff[L::Q];
    bool inbb[L::Q];
    row_links<L>(b, y, z, -1, inoff, inbb);
    const int64_t own_row = (int64_t)row * b.nx;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int x = threadIdx.x; x < b.nx; x += blockDim.x) {
        const uint32_t m = lm ? lm[own_row + x] : 0u;
        if (m & kSolidBit) continue;
        T g[L::Q];
        load_natural<L, T>(lat, b, x, own_row, inoff, inbb, odd != 0, m, g);
        double dn = 0.0;
#pragma unroll
        for (int q = 0; q < L::Q; ++q) {
            dn += double(g[q]);
#pragma unroll
            for (int d = 0; d < L::D; ++d) acc[1 + d] += L::e[q][d] * double(g[q]);
        }
        const double n = rho_ref + dn;
        acc[0] += n;
        if (!(n > 0.0) || !isfinite(n)) acc[4] += 1.0;
    }
    __shared__ double red[16][5];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double s = 0.0;
        for (int w = 0; w < nwaves; ++w) s += red[w][threadIdx.x];
        part[(int64_t)row * 5 + threadIdx.x] = s;
    }
}

// Second pass, one workgroup, fixed order: out[5] = sum over rows.
__global__ void __launch_bounds__(1024) k_totals_final(const double *__restrict__ part, int rows,
                                                       double *__restrict__ out) {
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int r = threadIdx.x; r < rows; r += blockDim.x)
#pragma unroll
        for (int k = 0; k < 5; ++k) acc[k] += part[(int64_t)r * 5 + k];
    __shared__ double red[16][5];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double s = 0.0;
        for (int w = 0; w < nwaves; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// ---------------------------------------------------------------------------
// host-side launchers (dispatch on lattice and storage type)
// ---------------------------------------------------------------------------
template <class L, typename T, bool O3, bool W, bool LOCAL>
hipError_t launch_plain(int scheme, int parity, void *a, void *b, const Box &box, const Coef<T> &c, int block,
                        hipStream_t s) {
    const dim3 grid(box.ny * box.nz), blk(block);
    if (scheme == LBM_SCHEME_PUSH)
        hipLaunchKernelGGL((k_push<L, T, O3, W, LOCAL>), grid, blk, 0, s, (const T *)a, (T *)b, box, c);
    else if (parity == 0)
        hipLaunchKernelGGL((k_aa_even<L, T, O3, W, LOCAL>), grid, blk, 0, s, (T *)a, box, c);
    else
        hipLaunchKernelGGL((k_aa_odd<L, T, O3, W, LOCAL>), grid, blk, 0, s, (T *)a, box, c);
    return hipGetLastError();
}

template <class L, typename T, bool O3, bool W>
hipError_t launch_step_w(int scheme, int parity, void *a, void *b, const Box &box, const Coef<T> &c, int block,
                         const uint32_t *lm, const double *F, bool local, hipStream_t s) {
    const dim3 grid(box.ny * box.nz), blk(block);
    if constexpr (L::O4) {  // the 41-velocity set: no link mask (41 links), no per-cell weights
        if (lm || local) return hipErrorInvalidValue;
    } else {
        if (lm) {
            const Force<T> f{{T(F[0]), T(F[1]), T(F[2])}};
            if (scheme == LBM_SCHEME_PUSH)
                hipLaunchKernelGGL((k_push_p<L, T, O3, W>), grid, blk, 0, s, (const T *)a, (T *)b, lm, box, c, f);
            else if (parity == 0)
                hipLaunchKernelGGL((k_aa_even_p<L, T, O3, W>), grid, blk, 0, s, (T *)a, lm, box, c, f);
            else
                hipLaunchKernelGGL((k_aa_odd_p<L, T, O3, W>), grid, blk, 0, s, (T *)a, lm, box, c, f);
            return hipGetLastError();
        }
        if (local) return launch_plain<L, T, O3, W, true>(scheme, parity, a, b, box, c, block, s);
    }
    return launch_plain<L, T, O3, W, false>(scheme, parity, a, b, box, c, block, s);
}

// 32-bit byte offsets while every slot of a lattice lies below 4 GiB from its base.
template <class L, typename T, bool O3>
hipError_t launch_step_o(int scheme, int parity, void *a, void *b, const Box &box, const Coef<T> &c, int block,
                         const uint32_t *lm, const double *F, bool local, hipStream_t s) {
    const bool wide = (uint64_t)L::Q * (uint64_t)box.plane * sizeof(T) >= (uint64_t(1) << 32);
    if (wide) return launch_step_w<L, T, O3, true>(scheme, parity, a, b, box, c, block, lm, F, local, s);
    return launch_step_w<L, T, O3, false>(scheme, parity, a, b, box, c, block, lm, F, local, s);
}

template <class L, typename T>
hipError_t launch_step_t(int scheme, int parity, void *a, void *b, const Box &box, const Model &m, double tau,
                         double rho_ref, int block, const uint32_t *lm, const double *F, hipStream_t s) {
    const Coef<T> c = make_coef<T>(m, tau, rho_ref);
    const bool local = m.local != 0;
    if (has_third_order(m)) return launch_step_o<L, T, true>(scheme, parity, a, b, box, c, block, lm, F, local, s);
    return launch_step_o<L, T, false>(scheme, parity, a, b, box, c, block, lm, F, local, s);
}

template <class L, typename T>
hipError_t launch_init_t(void *lat, const double *n0, const double *u0, const Box &box, const Model &m,
                         double tau, double rho_ref, int block, hipStream_t s) {
    const Coef<double> c = make_coef<double>(m, tau, rho_ref);
    const int o3 = has_third_order(m) ? 1 : 0;
    if constexpr (L::O4) {
        hipLaunchKernelGGL((k_init<L, T, false>), dim3(box.ny * box.nz), dim3(block), 0, s, (T *)lat, n0, u0, box, c,
                           o3);
    } else if (m.local) {
        hipLaunchKernelGGL((k_init<L, T, true>), dim3(box.ny * box.nz), dim3(block), 0, s, (T *)lat, n0, u0, box, c,
                           o3);
    } else {
        hipLaunchKernelGGL((k_init<L, T, false>), dim3(box.ny * box.nz), dim3(block), 0, s, (T *)lat, n0, u0, box,
                           c, o3);
    }
    return hipGetLastError();
}

template <class L, typename T>
hipError_t launch_moments_t(const void *lat, double *n, double *u, const Box &box, double rho_ref, int odd,
                            int block, const uint32_t *lm, const double *F, int row0, int nrows, int64_t ostride,
                            hipStream_t s) {
    const Force<double> f{{F ? F[0] : 0.0, F ? F[1] : 0.0, F ? F[2] : 0.0}};
    if (row0 < 0 || nrows < 1 || (int64_t)row0 + nrows > (int64_t)box.ny * box.nz || ostride < (int64_t)nrows * box.nx)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_moments<L, T>), dim3(nrows), dim3(block), 0, s, (const T *)lat, n, u, box, rho_ref, odd, lm,
                       f, row0, ostride);
    return hipGetLastError();
}

template <class L, typename T>
hipError_t launch_totals_t(const void *lat, double *part, double *out, const Box &box, double rho_ref, int odd,
                           int block, const uint32_t *lm, hipStream_t s) {
    const int rows = box.ny * box.nz;
    hipLaunchKernelGGL((k_totals_rows<L, T>), dim3(rows), dim3(block), 0, s, (const T *)lat, part, box, rho_ref,
                       odd, lm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(1024), 0, s, (const double *)part, rows, out);
    return hipGetLastError();
}

template <class L>
hipError_t launch_link_mask_t(const unsigned char *solid, uint32_t *lm, const Box &box, int block, hipStream_t s) {
    hipLaunchKernelGGL((k_link_mask<L>), dim3(box.ny * box.nz), dim3(block), 0, s, solid, lm, box);
    return hipGetLastError();
}

// Dispatch on the velocity set (lbm_lattice) and the storage type.
#define LBM_DISPATCH(LAT, FP64, CALL)                                                \
    do {                                                                             \
        if ((LAT) == LBM_D1V3) { if (FP64) { using L = D1Q3; using T = double; return CALL; } \
                                 else { using L = D1Q3; using T = float; return CALL; } }     \
        if ((LAT) == LBM_D2V9) { if (FP64) { using L = D2Q9; using T = double; return CALL; } \
                                 else { using L = D2Q9; using T = float; return CALL; } }     \
        if ((LAT) == LBM_D2V41) { if (FP64) { using L = D2Q41; using T = double; return CALL; } \
                                  else { using L = D2Q41; using T = float; return CALL; } }     \
        if (FP64) { using L = D3Q19; using T = double; return CALL; }                \
        else { using L = D3Q19; using T = float; return CALL; }                      \
    } while (0)

hipError_t launch_step(int lattice, int fp64, int scheme, int parity, void *a, void *b, const Box &box, const Model &m,
                       double tau, double rho_ref, int block, const uint32_t *lm, const double *F, hipStream_t s) {
    LBM_DISPATCH(lattice, fp64, (launch_step_t<L, T>(scheme, parity, a, b, box, m, tau, rho_ref, block, lm, F, s)));
}

hipError_t launch_init(int lattice, int fp64, void *lat, const double *n0, const double *u0, const Box &box,
                       const Model &m, double tau, double rho_ref, int block, hipStream_t s) {
    LBM_DISPATCH(lattice, fp64, (launch_init_t<L, T>(lat, n0, u0, box, m, tau, rho_ref, block, s)));
}

hipError_t launch_moments(int lattice, int fp64, const void *lat, double *n, double *u, const Box &box, double rho_ref,
                          int odd, int block, const uint32_t *lm, const double *F, int row0, int nrows,
                          int64_t ostride, hipStream_t s) {
    LBM_DISPATCH(lattice, fp64,
                 (launch_moments_t<L, T>(lat, n, u, box, rho_ref, odd, block, lm, F, row0, nrows, ostride, s)));
}

hipError_t launch_totals(int lattice, int fp64, const void *lat, double *part, double *out, const Box &box,
                         double rho_ref, int odd, int block, const uint32_t *lm, hipStream_t s) {
    LBM_DISPATCH(lattice, fp64, (launch_totals_t<L, T>(lat, part, out, box, rho_ref, odd, block, lm, s)));
}

hipError_t launch_link_mask(int D, const unsigned char *solid, uint32_t *lm, const Box &box, int block,
                            hipStream_t s) {
    if (D == 1) return launch_link_mask_t<D1Q3>(solid, lm, box, block, s);
    if (D == 2) return launch_link_mask_t<D2Q9>(solid, lm, box, block, s);
    return launch_link_mask_t<D3Q19>(solid, lm, box, block, s);
}

}  // namespace lbm
