// Batched sweep of many independent closed shock tubes (nx x 4 cells, halfway
// bounce-back walls in x, periodic in y, d2v9), each with its own length,
// relaxation time and number of steps, advanced by LDS-resident temporal
// blocking.
//
// A tile is a run of `s` columns of one tube.  A workgroup loads the tile plus
// up to H halo columns on each side (all 4 rows, all 9 populations) from global
// memory into LDS, advances h <= H lattice BGK steps there in place with the AA
// pattern, and writes the tile's own columns back.  The edges of the loaded
// window are treated as bounce-back walls: at the tube's real walls that is the
// boundary condition, and at a cut through the tube the wrong reflection only
// reaches h columns into the halo in h steps (one column per step), never the
// tile itself.  Rounds of H steps alternate between two global buffers; a tube
// finished before the others simply drops out of later rounds (tiles are ordered
// by the number of rounds of their tube, so each round's active tiles are a
// prefix of the tile list).
//
// Every cell update is the same collide() as the plain field kernels, so a tube
// advanced here is bit-for-bit the tube advanced by lbm_step on an nx x 4 box.
// Global traffic per lattice update drops by the factor of about H, and the
// sweep is bound by LDS bandwidth and arithmetic rather than by HBM.
#include <hip/hip_runtime.h>

#include "lbm_batch.h"
#include "lbm_collide.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr int NY = 4;  // rows of every tube
constexpr int kTubeThreads = 1024;  // per-tube kernels: one workgroup per tube
using Lat = D2Q9;

// LDS window layout: lds[(q * 4 + y) * WP + c], WP a power of two >= W (the
// row stride, a template parameter so that cell -> (row, column) is a shift and
// a mask).  Columns c >= W of a row are unused.
//
// Natural-layout populations of cell (y, c): after an even number of AA steps
// they sit in their own slots; after an odd number, g_a of the cell is in the
// slot of -a at c - e_a (its own slot a where that crosses a window edge, which
// is a wall).  EDGE selects the wall checks (only the first and last column of
// the window need them).
// Row-and-column bases of the rows y - 1, y, y + 1 (periodic in y); every
// population's slot is one of them plus a compile-time offset (plane and x
// shift), which the LDS instructions take as an immediate.
template <int WP>
struct RowBases {
    int m, z, p;  // (y-1) WP + c, y WP + c, (y+1) WP + c
    __device__ __forceinline__ RowBases(int y, int c)
        : m(((y - 1) & (NY - 1)) * WP + c), z(y * WP + c), p(((y + 1) & (NY - 1)) * WP + c) {}
    __device__ __forceinline__ int row(int dy) const { return dy < 0 ? m : (dy > 0 ? p : z); }
};

template <int WP, typename T, bool EDGE>
__device__ __forceinline__ void load_cell(const T *__restrict__ lds, int W, int y, int c, bool odd,
                                          T (&g)[Lat::Q]) {
    constexpr int pl = NY * WP;
    if (!odd) {
#pragma unroll
        for (int q = 0; q < Lat::Q; ++q) g[q] = lds[q * pl + y * WP + c];
    } else if (!EDGE) {
        const RowBases<WP> rb(y, c);
#pragma unroll
        for (int q = 0; q < Lat::Q; ++q)  // from the slot of -q at (y - e_y, c - e_x)
            g[q] = lds[rb.row(-Lat::e[q][1]) + (Lat::opp[q] * pl - Lat::e[q][0])];
    } else {
#pragma unroll
        for (int q = 0; q < Lat::Q; ++q) {
            const int cs = c - Lat::e[q][0];
            const int ys = (y - Lat::e[q][1]) & (NY - 1);
            if (EDGE && (cs < 0 || cs >= W)) g[q] = lds[q * pl + y * WP + c];
            else g[q] = lds[Lat::opp[q] * pl + ys * WP + cs];
        }
    }
}

template <int WP, typename T, bool EDGE>
__device__ __forceinline__ void store_cell(T *__restrict__ lds, int W, int y, int c, bool odd, const T (&g)[Lat::Q]) {
    constexpr int pl = NY * WP;
    if (!odd) {
#pragma unroll
        for (int q = 0; q < Lat::Q; ++q) lds[Lat::opp[q] * pl + y * WP + c] = g[q];
    } else if (!EDGE) {
        const RowBases<WP> rb(y, c);
#pragma unroll
        for (int q = 0; q < Lat::Q; ++q)  // to slot q at (y + e_y, c + e_x)
            lds[rb.row(Lat::e[q][1]) + (q * pl + Lat::e[q][0])] = g[q];
    } else {
#pragma unroll
        for (int q = 0; q < Lat::Q; ++q) {
            const int xt = c + Lat::e[q][0];
            const int yt = (y + Lat::e[q][1]) & (NY - 1);
            if (EDGE && (xt < 0 || xt >= W)) lds[Lat::opp[q] * pl + y * WP + c] = g[q];
            else lds[q * pl + yt * WP + xt] = g[q];
        }
    }
}

// One round: each workgroup takes one tile of the active prefix, or, with a
// tile list (list[0] tiles, their indices from list[1]), the tile the list
// names for it (workgroups past the list's count return at once).  The window
// holds W = s + halo columns (W <= WP); thread t handles the cells
// t, t + blockDim, ... of the 4 x WP cell grid (row = cell / WP).
template <int WP, typename T, bool O3>
__global__ void __launch_bounds__(1024) k_batch_round(T *__restrict__ buf0, T *__restrict__ buf1,
                                                      const BatchTube *__restrict__ tubes,
                                                      const BatchTile *__restrict__ tiles,
                                                      const int *__restrict__ list, int round, int H, Coef<T> c) {
    static_assert(WP % 64 == 0, "a wavefront's 64 cells must lie in one window row");
    __shared__ T lds[Lat::Q * NY * WP];
    constexpr int CELLS = NY * WP;
    int ti = blockIdx.x;
    if (list) {
        if (ti >= list[0]) return;
        ti = list[1 + ti];
    }
    const BatchTile tl = tiles[ti];
    const BatchTube tb = tubes[tl.tube];
    int h = tb.steps - round * H;
    if (h > H) h = H;
    if (h <= 0) return;
    // buffers: the tube's state is in buffer (cur ^ (round & 1)) at the start of this round
    const int from = tb.cur ^ (round & 1);
    const T *__restrict__ src = from ? buf1 : buf0;
    T *__restrict__ dst = from ? buf0 : buf1;
    c.omega = T(tb.omega);

    const int hl = tl.x0 < h ? tl.x0 : h;
    const int right = tb.nx - tl.x0 - tl.s;
    const int hr = right < h ? right : h;
    const int w0 = tl.x0 - hl;
    const int W = tl.s + hl + hr;
    const int64_t gpl = (int64_t)NY * tb.nx;
    const T *__restrict__ gsrc = src + tb.off + w0;
    T *__restrict__ gdst = dst + tb.off + w0;

    // load the window (natural layout), coalesced along x
    for (int i = threadIdx.x; i < Lat::Q * CELLS; i += blockDim.x) {
        const int qy = i / WP, x = i & (WP - 1);
        if (x < W) lds[i] = gsrc[(int64_t)(qy >> 2) * gpl + (int64_t)(qy & 3) * tb.nx + x];
    }
    __syncthreads();

    // The wall checks concern only odd steps (even steps use the cell's own
    // slots) and only the window's first and last columns.  The choice is made
    // per wavefront (its 64 cells lie in one row, WP being a multiple of 64), so
    // that a wavefront runs one path: a per-lane branch made the two wavefronts
    // of a row that hold an end column run the whole collision twice.
    for (int step = 0; step < h; ++step) {
        const bool odd = step & 1;
        for (int cell = threadIdx.x; cell < CELLS; cell += blockDim.x) {
            const int y = cell / WP, x = cell & (WP - 1);
            const int x0 = __builtin_amdgcn_readfirstlane(x - (int)(threadIdx.x & 63));  // the wavefront's first column
            if (x >= W) continue;
            T g[Lat::Q];
            if (!odd) {
                load_cell<WP, T, false>(lds, W, y, x, false, g);
                collide<Lat, T, O3>(g, c);
                store_cell<WP, T, false>(lds, W, y, x, false, g);
            } else if (x0 > 0 && x0 + 63 < W - 1) {
                load_cell<WP, T, false>(lds, W, y, x, true, g);
                collide<Lat, T, O3>(g, c);
                store_cell<WP, T, false>(lds, W, y, x, true, g);
            } else {
                load_cell<WP, T, true>(lds, W, y, x, true, g);
                collide<Lat, T, O3>(g, c);
                store_cell<WP, T, true>(lds, W, y, x, true, g);
            }
        }
        __syncthreads();
    }

    // write the tile's own columns back in natural layout
    const bool odd_end = h & 1;
    for (int cell = threadIdx.x; cell < CELLS; cell += blockDim.x) {
        const int y = cell / WP, x = cell & (WP - 1);
        if (x < hl || x >= hl + tl.s) continue;
        T g[Lat::Q];
        load_cell<WP, T, true>(lds, W, y, x, odd_end, g);
#pragma unroll
        for (int q = 0; q < Lat::Q; ++q) gdst[(int64_t)q * gpl + (int64_t)y * tb.nx + x] = g[q];
    }
}

// Initial populations of every tube: equilibrium at rest with n_left for
// x < nx/2 and n_right beyond (f = f_eq(n, 0), g = w (n - rho_ref)).
template <typename T>
__global__ void __launch_bounds__(256) k_batch_init(T *__restrict__ buf0, T *__restrict__ buf1,
                                                    const BatchTube *__restrict__ tubes, Coef<double> c) {
    const BatchTube tb = tubes[blockIdx.x];
    T *__restrict__ g = (tb.cur ? buf1 : buf0) + tb.off;
    const int64_t gpl = (int64_t)NY * tb.nx;
    for (int i = threadIdx.x; i < NY * tb.nx; i += blockDim.x) {
        const int x = i % tb.nx;
        const double n = x < tb.nx / 2 ? tb.n_left : tb.n_right;
        const double dn = n - c.rho_ref;
#pragma unroll
        for (int q = 0; q < Lat::Q; ++q) g[q * gpl + i] = T(c.w[Lat::cls[q]] * dn);
    }
}

// Populations of the masked tubes set to equilibrium with the given packed
// float64 fields (n[cells], u[2][cells], cells in tube order, x fastest).
template <typename T>
__global__ void __launch_bounds__(256) k_batch_set_eq(T *__restrict__ buf0, T *__restrict__ buf1,
                                                      const BatchTube *__restrict__ tubes,
                                                      const unsigned char *__restrict__ mask,
                                                      const double *__restrict__ n_in, const double *__restrict__ u_in,
                                                      int64_t total_cells, Coef<double> c) {
    const BatchTube tb = tubes[blockIdx.x];
    if (!mask[blockIdx.x]) return;
    T *__restrict__ g = (tb.cur ? buf1 : buf0) + tb.off;
    const int64_t gpl = (int64_t)NY * tb.nx;
    const int64_t cell0 = tb.off / Lat::Q;
    for (int i = threadIdx.x; i < NY * tb.nx; i += blockDim.x) {
        const double n = n_in[cell0 + i];
        const double ux = u_in[cell0 + i], uy = u_in[total_cells + cell0 + i];
        const double u2 = ux * ux + uy * uy;
        const double dn = n - c.rho_ref;
#pragma unroll
        for (int q = 0; q < Lat::Q; ++q) {
            const int k = Lat::cls[q];
            const double eu = Lat::e[q][0] * ux + Lat::e[q][1] * uy;
            const double sm1 = eu * (c.l1[k] + c.c3[k] * u2 + c.k4[k] * eu * eu) + c.q[k] * eu * eu + c.s[k] * u2;
            g[q * gpl + i] = T(c.w[k] * (dn + n * sm1));
        }
    }
}

// Row-averaged float32 profiles of tubes of equal length: prof[t][0][x] = mean_y n,
// prof[t][1][x] = mean_y u_x (the rows of a tube started at rest with a step in x
// stay identical; the mean is taken all the same).
// Tubes with skip[t] set (skip may be null) are left out: their profiles are kept.
template <typename T>
__global__ void __launch_bounds__(1024) k_batch_profiles(const T *__restrict__ buf0, const T *__restrict__ buf1,
                                                        const BatchTube *__restrict__ tubes, float *__restrict__ prof,
                                                        double rho_ref, const unsigned char *__restrict__ skip) {
    if (skip && skip[blockIdx.x]) return;
    const BatchTube tb = tubes[blockIdx.x];
    const T *__restrict__ g = (tb.cur ? buf1 : buf0) + tb.off;
    const int64_t gpl = (int64_t)NY * tb.nx;
    float *pn = prof + (int64_t)blockIdx.x * 2 * tb.nx;
    for (int x = threadIdx.x; x < tb.nx; x += blockDim.x) {
        double ns = 0.0, us = 0.0;
        for (int y = 0; y < NY; ++y) {
            double dn = 0.0, jx = 0.0;
#pragma unroll
            for (int q = 0; q < Lat::Q; ++q) {
                const double v = double(g[q * gpl + (int64_t)y * tb.nx + x]);
                dn += v;
                jx += Lat::e[q][0] * v;
            }
            const double n = rho_ref + dn;
            ns += n;
            us += jx / n;
        }
        pn[x] = float(ns / NY);
        pn[tb.nx + x] = float(us / NY);
    }
}

// The populations of one tube (planes gpl apart) set to f = f_eq(n(x), (u(x), 0))
// on every row from its float32 profile pn = (n[nx], u[nx]), in float64.
template <typename T>
__device__ __forceinline__ void set_from_profile(T *__restrict__ g, int64_t gpl, int nx, const float *__restrict__ pn,
                                                 const Coef<double> &c) {
    for (int i = threadIdx.x; i < NY * nx; i += blockDim.x) {
        const int x = i % nx;
        const double n = pn[x], ux = pn[nx + x];
        const double u2 = ux * ux, dn = n - c.rho_ref;
#pragma unroll
        for (int q = 0; q < Lat::Q; ++q) {
            const int k = Lat::cls[q];
            const double eu = Lat::e[q][0] * ux;
            const double sm1 = eu * (c.l1[k] + c.c3[k] * u2 + c.k4[k] * eu * eu) + c.q[k] * eu * eu + c.s[k] * u2;
            g[q * gpl + i] = T(c.w[k] * (dn + n * sm1));
        }
    }
}

// Masked tubes set to f = f_eq(n(x), (u(x), 0)) on every row from float32 profiles.
template <typename T>
__global__ void __launch_bounds__(1024) k_batch_set_profiles(T *__restrict__ buf0, T *__restrict__ buf1,
                                                            const BatchTube *__restrict__ tubes,
                                                            const unsigned char *__restrict__ mask,
                                                            const float *__restrict__ prof, Coef<double> c) {
    const BatchTube tb = tubes[blockIdx.x];
    if (!mask[blockIdx.x]) return;
    T *__restrict__ g = (tb.cur ? buf1 : buf0) + tb.off;
    const int64_t gpl = (int64_t)NY * tb.nx;
    set_from_profile(g, gpl, tb.nx, prof + (int64_t)blockIdx.x * 2 * tb.nx, c);
}

// Per tube after a device decision (mask[t] = 1: accepted), for a hybrid run
// that keeps an accepted tube's state as its profile until a lattice step needs
// it (lazy[t] = 1: the tube's state is pin[t], its populations are stale):
// accepted, pin[t] = pout[t] and lazy[t] = 1; rejected with lazy[t] = 1, its
// populations are set from pin[t] (its state when the jump began) and lazy[t] = 0.
template <typename T>
__global__ void __launch_bounds__(1024) k_batch_commit(T *__restrict__ buf0, T *__restrict__ buf1,
                                                      const BatchTube *__restrict__ tubes,
                                                      const unsigned char *__restrict__ mask,
                                                      unsigned char *__restrict__ lazy, float *__restrict__ pin,
                                                      const float *__restrict__ pout, Coef<double> c) {
    const int t = blockIdx.x;
    const BatchTube tb = tubes[t];
    const bool acc = mask[t], was_lazy = lazy[t];
    __syncthreads();  // every thread has read lazy[t]
    const int64_t np = 2 * (int64_t)tb.nx, o = (int64_t)t * np;
    if (acc) {
        for (int64_t i = threadIdx.x; i < np; i += blockDim.x) pin[o + i] = pout[o + i];
        if (threadIdx.x == 0) lazy[t] = 1;
    } else if (was_lazy) {
        set_from_profile((tb.cur ? buf1 : buf0) + tb.off, (int64_t)NY * tb.nx, tb.nx, pin + o, c);
        if (threadIdx.x == 0) lazy[t] = 0;
    }
}

__global__ void __launch_bounds__(256) k_clear_bytes(unsigned char *__restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Moments of every tube into packed float64 fields and, per tube, the number of
// cells whose density is not finite and positive.
template <typename T>
__global__ void __launch_bounds__(256) k_batch_moments(const T *__restrict__ buf0, const T *__restrict__ buf1,
                                                       const BatchTube *__restrict__ tubes, double *__restrict__ n_out,
                                                       double *__restrict__ u_out, int *__restrict__ bad,
                                                       int64_t total_cells, double rho_ref) {
    const BatchTube tb = tubes[blockIdx.x];
    const T *__restrict__ g = (tb.cur ? buf1 : buf0) + tb.off;
    const int64_t gpl = (int64_t)NY * tb.nx;
    const int64_t cell0 = tb.off / Lat::Q;
    int nbad = 0;
    for (int i = threadIdx.x; i < NY * tb.nx; i += blockDim.x) {
        double dn = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
        for (int q = 0; q < Lat::Q; ++q) {
            const double v = double(g[q * gpl + i]);
            dn += v;
            jx += Lat::e[q][0] * v;
            jy += Lat::e[q][1] * v;
        }
        const double n = rho_ref + dn;
        if (!(n > 0.0) || !isfinite(n) || !isfinite(jx) || !isfinite(jy)) ++nbad;
        if (n_out) {
            n_out[cell0 + i] = n;
            u_out[cell0 + i] = jx / n;
            u_out[total_cells + cell0 + i] = jy / n;
        }
    }
    __shared__ int red[4];
    int v = nbad;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) bad[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// After a schedule: the state of a tube that ran an odd number of rounds is in
// the other buffer.
__global__ void __launch_bounds__(256) k_batch_flip(BatchTube *__restrict__ tubes, int ntubes, int H) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntubes) return;
    const int rounds = (tubes[t].steps + H - 1) / H;
    if (rounds & 1) tubes[t].cur ^= 1;
}

// A device-decided schedule from per-tube indicators (one workgroup of 1024
// threads): a tube is accepted when its indicator is finite and <= tol, then
// mask[t] = 1 and it takes no steps, else it takes nsteps; *count = the number
// rejected; the tiles of the rejected tubes, in tile order, go into list[1..]
// with their count in list[0] (1024 tiles per pass).
__device__ __forceinline__ bool accepted(const float *resid, int t, float tol) {
    const float r = resid[t];
    return isfinite(r) && r <= tol;
}
__global__ void __launch_bounds__(1024) k_batch_decide_list(const float *__restrict__ resid, int ntubes, float tol,
                                                            int nsteps, unsigned char *__restrict__ mask,
                                                            BatchTube *__restrict__ tubes,
                                                            const BatchTile *__restrict__ tiles, int ntiles,
                                                            int *__restrict__ list, int *__restrict__ count) {
    __shared__ int wsum[16];  // per wavefront: rejected tubes, then flagged tiles of a pass
    __shared__ int base;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const unsigned long long below = lane ? ~0ull >> (64 - lane) : 0ull;  // the lanes before this one
    int nrej = 0;
    for (int t = threadIdx.x; t < ntubes; t += blockDim.x) {
        const bool ok = accepted(resid, t, tol);
        mask[t] = ok;
        tubes[t].steps = ok ? 0 : nsteps;
        nrej += !ok;
    }
    for (int o = 32; o > 0; o >>= 1) nrej += __shfl_xor(nrej, o);
    if (lane == 0) wsum[wave] = nrej;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < nw; ++w) tot += wsum[w];
        *count = tot;
        base = 0;
    }
    __syncthreads();
    // the flagged tiles of a pass in tile order: a wavefront's by the ballot of
    // its lanes, the wavefronts' in order by their counts
    for (int i0 = 0; i0 < ntiles; i0 += blockDim.x) {
        const int i = i0 + (int)threadIdx.x;
        const bool flag = i < ntiles && !accepted(resid, tiles[i].tube, tol);
        const unsigned long long m = __builtin_amdgcn_ballot_w64(flag);
        if (lane == 0) wsum[wave] = __popcll(m);
        __syncthreads();
        int before = base;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (flag) list[1 + before + __popcll(m & below)] = i;
        __syncthreads();  // every thread has read wsum and base
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w = 0; w < nw; ++w) tot += wsum[w];
            base += tot;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) list[0] = base;
}

// The step counts of a schedule written into the tube table.
__global__ void __launch_bounds__(256) k_batch_set_steps(BatchTube *__restrict__ tubes, int ntubes,
                                                         const int *__restrict__ steps) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntubes) tubes[t].steps = steps[t];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int WP, typename T>
hipError_t batch_round_wp(void *b0, void *b1, const BatchTube *tubes, const BatchTile *tiles, const int *list,
                          int ntiles, int round, int H, int block, const Coef<T> &c, bool o3, hipStream_t s) {
    if (o3)
        hipLaunchKernelGGL((k_batch_round<WP, T, true>), dim3(ntiles), dim3(block), 0, s, (T *)b0, (T *)b1, tubes,
                           tiles, list, round, H, c);
    else
        hipLaunchKernelGGL((k_batch_round<WP, T, false>), dim3(ntiles), dim3(block), 0, s, (T *)b0, (T *)b1, tubes,
                           tiles, list, round, H, c);
    return hipGetLastError();
}

// The window stride: the smallest power of two that holds W columns.
template <typename T>
hipError_t batch_round_t(void *b0, void *b1, const BatchTube *tubes, const BatchTile *tiles, const int *list,
                         int ntiles, int round, int H, int W, int block, const Model &m, double rho_ref,
                         hipStream_t s) {
    const Coef<T> c = make_coef<T>(m, 1.0, rho_ref);
    const bool o3 = has_third_order(m);
    if (W <= 128) return batch_round_wp<128, T>(b0, b1, tubes, tiles, list, ntiles, round, H, block, c, o3, s);
    if (W <= 256) return batch_round_wp<256, T>(b0, b1, tubes, tiles, list, ntiles, round, H, block, c, o3, s);
    if (W <= 512) return batch_round_wp<512, T>(b0, b1, tubes, tiles, list, ntiles, round, H, block, c, o3, s);
    return hipErrorInvalidValue;
}

hipError_t batch_round(int fp64, void *b0, void *b1, const BatchTube *tubes, const BatchTile *tiles, const int *list,
                       int ntiles, int round, int H, int W, int block, const Model &m, double rho_ref, hipStream_t s) {
    if (fp64) return batch_round_t<double>(b0, b1, tubes, tiles, list, ntiles, round, H, W, block, m, rho_ref, s);
    return batch_round_t<float>(b0, b1, tubes, tiles, list, ntiles, round, H, W, block, m, rho_ref, s);
}

hipError_t batch_decide_list(const float *resid, int ntubes, float tol, int nsteps, unsigned char *mask,
                             BatchTube *tubes, const BatchTile *tiles, int ntiles, int *list, int *count,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_batch_decide_list, dim3(1), dim3(1024), 0, s, resid, ntubes, tol, nsteps, mask, tubes, tiles,
                       ntiles, list, count);
    return hipGetLastError();
}

hipError_t batch_set_steps(BatchTube *tubes, int ntubes, const int *steps, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_set_steps, dim3((ntubes + 255) / 256), dim3(256), 0, s, tubes, ntubes, steps);
    return hipGetLastError();
}

hipError_t batch_flip(BatchTube *tubes, int ntubes, int H, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_flip, dim3((ntubes + 255) / 256), dim3(256), 0, s, tubes, ntubes, H);
    return hipGetLastError();
}

hipError_t batch_init(int fp64, void *b0, void *b1, const BatchTube *tubes, int ntubes, const Model &m,
                      double rho_ref, hipStream_t s) {
    const Coef<double> c = make_coef<double>(m, 1.0, rho_ref);
    if (fp64) hipLaunchKernelGGL(k_batch_init<double>, dim3(ntubes), dim3(256), 0, s, (double *)b0, (double *)b1, tubes, c);
    else hipLaunchKernelGGL(k_batch_init<float>, dim3(ntubes), dim3(256), 0, s, (float *)b0, (float *)b1, tubes, c);
    return hipGetLastError();
}

hipError_t batch_set_eq(int fp64, void *b0, void *b1, const BatchTube *tubes, int ntubes, const unsigned char *mask,
                        const double *n, const double *u, int64_t total_cells, const Model &m, double rho_ref,
                        hipStream_t s) {
    const Coef<double> c = make_coef<double>(m, 1.0, rho_ref);
    if (fp64)
        hipLaunchKernelGGL(k_batch_set_eq<double>, dim3(ntubes), dim3(256), 0, s, (double *)b0, (double *)b1, tubes,
                           mask, n, u, total_cells, c);
    else
        hipLaunchKernelGGL(k_batch_set_eq<float>, dim3(ntubes), dim3(256), 0, s, (float *)b0, (float *)b1, tubes,
                           mask, n, u, total_cells, c);
    return hipGetLastError();
}

hipError_t batch_profiles(int fp64, const void *b0, const void *b1, const BatchTube *tubes, int ntubes, float *prof,
                          double rho_ref, hipStream_t s, const unsigned char *skip) {
    if (fp64)
        hipLaunchKernelGGL(k_batch_profiles<double>, dim3(ntubes), dim3(kTubeThreads), 0, s, (const double *)b0,
                           (const double *)b1, tubes, prof, rho_ref, skip);
    else
        hipLaunchKernelGGL(k_batch_profiles<float>, dim3(ntubes), dim3(kTubeThreads), 0, s, (const float *)b0,
                           (const float *)b1, tubes, prof, rho_ref, skip);
    return hipGetLastError();
}

hipError_t batch_commit(int fp64, void *b0, void *b1, const BatchTube *tubes, int ntubes, const unsigned char *mask,
                        unsigned char *lazy, float *pin, const float *pout, const Model &m, double rho_ref,
                        hipStream_t s) {
    const Coef<double> c = make_coef<double>(m, 1.0, rho_ref);
    if (fp64)
        hipLaunchKernelGGL(k_batch_commit<double>, dim3(ntubes), dim3(kTubeThreads), 0, s, (double *)b0,
                           (double *)b1, tubes, mask, lazy, pin, pout, c);
    else
        hipLaunchKernelGGL(k_batch_commit<float>, dim3(ntubes), dim3(kTubeThreads), 0, s, (float *)b0,
                           (float *)b1, tubes, mask, lazy, pin, pout, c);
    return hipGetLastError();
}

hipError_t clear_bytes(unsigned char *p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_bytes, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t batch_set_profiles(int fp64, void *b0, void *b1, const BatchTube *tubes, int ntubes,
                              const unsigned char *mask, const float *prof, const Model &m, double rho_ref,
                              hipStream_t s) {
    const Coef<double> c = make_coef<double>(m, 1.0, rho_ref);
    if (fp64)
        hipLaunchKernelGGL(k_batch_set_profiles<double>, dim3(ntubes), dim3(kTubeThreads), 0, s, (double *)b0,
                           (double *)b1, tubes, mask, prof, c);
    else
        hipLaunchKernelGGL(k_batch_set_profiles<float>, dim3(ntubes), dim3(kTubeThreads), 0, s, (float *)b0,
                           (float *)b1, tubes, mask, prof, c);
    return hipGetLastError();
}

hipError_t batch_moments(int fp64, const void *b0, const void *b1, const BatchTube *tubes, int ntubes, double *n,
                         double *u, int *bad, int64_t total_cells, double rho_ref, hipStream_t s) {
    if (fp64)
        hipLaunchKernelGGL(k_batch_moments<double>, dim3(ntubes), dim3(256), 0, s, (const double *)b0,
                           (const double *)b1, tubes, n, u, bad, total_cells, rho_ref);
    else
        hipLaunchKernelGGL(k_batch_moments<float>, dim3(ntubes), dim3(256), 0, s, (const float *)b0,
                           (const float *)b1, tubes, n, u, bad, total_cells, rho_ref);
    return hipGetLastError();
}

}  // namespace lbm
