// Kernels of the 1D convolutional surrogate: forward, backward and Adam.
//
// Network: features (n-1)/0.25, u/0.25, (tau-0.75)/0.25 -> conv 3->64 (dilation 1)
// -> GELU -> conv 64->64 (d 3) -> GELU -> conv 64->64 (d 9) -> GELU -> conv 64->2
// (d 27) = y;  n' = n + 0.25 y0, u' = u + 0.25 y1.  Kernel 5, zero padding.
// conv(a)[x, co] = b[co] + sum_{tap, ci} W[tap][co][ci] a[x + (tap-2) d, ci].
//
// Storage: activations bfloat16, channels last ([B][L][64]); weights bfloat16
// (from float32 master copies), accumulation float32.  The two 64->64 layers
// (97% of the flops) run on the bf16 matrix cores: a workgroup computes a 64
// (positions) x 64 (channels) tile as four 32x32 blocks, one per wavefront, with
// v_mfma_f32_32x32x16_bf16 over K = 5 taps x 64 channels.  The data-gradient of
// a layer is the same kernel with the taps reversed and the weights transposed;
// the weight-gradient is a K = positions reduction, per workgroup into float32
// partials that a second kernel sums in a fixed order.  The 3->64 and 64->2
// layers are too thin for the matrix cores and use plain FMA.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <type_traits>

namespace srg {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int CH = 64;
constexpr int KT = 5;
constexpr float FS = 0.25f;       // feature scale
constexpr float TAU_C = 0.75f;    // tau centre

// erf by Abramowitz & Stegun, Handbook of Mathematical Functions (1964), formula
// 7.1.26 (Hastings' approximation): for x >= 0,
//   erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2),  t = 1 / (1 + p x),
// with an absolute error of at most 1.5e-7 (far below the bfloat16 rounding the
// activations then take); odd extension for x < 0.  exp(-x^2) is shared with GELU'.
struct ErfExp {
    float erf, e;  // erf(x) and exp(-x^2)
};
__device__ __forceinline__ ErfExp erf_exp(float x) {
    const float ax = __builtin_fabsf(x);
    const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f, ax, 1.0f));
    float p = __builtin_fmaf(1.061405429f, t, -1.453152027f);
    p = __builtin_fmaf(p, t, 1.421413741f);
    p = __builtin_fmaf(p, t, -0.284496736f);
    p = __builtin_fmaf(p, t, 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(-ax * ax * 1.4426950408889634f);
    const float r = __builtin_fmaf(-p * t, e, 1.0f);
    return {__builtin_copysignf(r, x), e};
}
// GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2
__device__ __forceinline__ float gelu(float z) {
    return 0.5f * z * (1.0f + erf_exp(z * 0.70710678118654752f).erf);
}
// GELU'(z) = Phi(z) + z phi(z), phi(z) = exp(-z^2 / 2) / sqrt(2 pi)
__device__ __forceinline__ float gelu_grad(float z) {
    const ErfExp q = erf_exp(z * 0.70710678118654752f);
    return __builtin_fmaf(z * 0.39894228040143268f, q.e, 0.5f * (1.0f + q.erf));
}
__device__ __forceinline__ __bf16 to_bf(float v) { return (__bf16)v; }
__device__ __forceinline__ float to_f(__bf16 v) { return (float)v; }

// bf16(GELU(z)) for a bfloat16 z by table: the forward rounds z to bfloat16
// before the GELU, so the result is a function of 16 bits.  A table covers the
// NE biased exponents E0 .. E0 + NE - 1 of both signs (2 NE 128 entries) and is
// written by gelu() itself, so a lookup gives the bits the computation gives;
// values outside it (smaller or larger magnitudes, zero, non-finite) are
// computed.  GeluT16: |z| in [2^-12, 16), 4096 entries, 8 KB of LDS (the layer-1
// kernel); GeluT32: |z| in [2^-24, 128), 8192 entries, 16 KB (the fused kernel,
// where a wavefront takes the computed path for all its values as soon as one
// lane holds a value outside the table: with the trained weights about 1 % of
// the pre-activations of layers 1-2 lie below 2^-12, and on strong shocks up to
// 17 % of layer 3's reach 16 and beyond (up to 62), so that with the smaller
// table nearly every wavefront took that path).
template <int E0, int NE>
struct GeluTable {
    static constexpr int HALF = NE * 128, N = 2 * HALF, BIAS = E0 << 7;
    static_assert(HALF == 0x800 || HALF == 0x1000, "the index's sign bit is bit 11 or 12");
    static __device__ __forceinline__ unsigned short entry(int i) {
        const unsigned bits = ((unsigned)(i / HALF) << 15) | (unsigned)((E0 << 7) + i % HALF);
        const __bf16 z = __builtin_bit_cast(__bf16, (unsigned short)bits);
        return __builtin_bit_cast(unsigned short, to_bf(gelu(to_f(z))));
    }
    static __device__ __forceinline__ bool lookup(__bf16 z, unsigned *index) {
        const unsigned bits = __builtin_bit_cast(unsigned short, z);
        const unsigned t = (bits & 0x7fffu) - (unsigned)(E0 << 7);
        *index = t + (bits >> 15) * HALF;
        return t < (unsigned)HALF;
    }
};
using GeluT16 = GeluTable<115, 16>;
using GeluT32 = GeluTable<103, 32>;

// GELU of bfloat16 pairs (32-bit words, low half first) by table, the index
// formed by 16-bit packed operations: per half t = (z & 0x7fff) - (E0 << 7), in
// the table when t < HALF, entry t + HALF sign.
typedef unsigned short us2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_bf2(float x, float y) {
    const bf16x2 v = {to_bf(x), to_bf(y)};
    return __builtin_bit_cast(unsigned, v);
}
// t of both halves
template <class Tab>
__device__ __forceinline__ unsigned gelu_bf2_t(unsigned z) {
    return __builtin_bit_cast(unsigned, __builtin_bit_cast(us2, z & 0x7fff7fffu) - (us2)((unsigned short)Tab::BIAS));
}
// v[i] from the table for every value, every read issued before any result is
// used; the index is taken within the table, so a value outside it reads some
// entry and must be replaced (gelu_bf2_outside, gelu_bf2_word)
template <class Tab, int N>
__device__ __forceinline__ void gelu_bf2_table(const unsigned (&z)[N], unsigned (&v)[N], const unsigned short *tab) {
    constexpr unsigned H = Tab::HALF;
    constexpr unsigned LOW = (H - 1u) * 0x10001u;  // t within the table
    constexpr unsigned SIGN = H * 0x10001u;        // the index's sign bit
    constexpr unsigned SH = H == 0x800 ? 4u : 3u;  // bit 15 -> that bit
    const char *tb = reinterpret_cast<const char *>(tab);
    us2 e[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const unsigned idx = (gelu_bf2_t<Tab>(z[i]) & LOW) | ((z[i] >> SH) & SIGN);
        const unsigned off = __builtin_bit_cast(unsigned, __builtin_bit_cast(us2, idx) << (us2)(1));
        e[i].x = *reinterpret_cast<const unsigned short *>(tb + (off & 0xffffu));
        e[i].y = *reinterpret_cast<const unsigned short *>(tb + (off >> 16));
    }
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = __builtin_bit_cast(unsigned, e[i]);
}
// nonzero when some value of z lies outside the table
template <class Tab, int N>
__device__ __forceinline__ unsigned gelu_bf2_outside(const unsigned (&z)[N]) {
    unsigned any = 0u;
#pragma unroll
    for (int i = 0; i < N; ++i) any |= gelu_bf2_t<Tab>(z[i]);
    return any & ((0x10000u - Tab::HALF) * 0x10001u);
}
// one word, each half from the table or computed
template <class Tab>
__device__ __forceinline__ unsigned gelu_bf2_word(unsigned z, const unsigned short *tab) {
    unsigned short r[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const __bf16 zh = __builtin_bit_cast(__bf16, (unsigned short)(z >> (16 * h)));
        unsigned idx;
        r[h] = Tab::lookup(zh, &idx) ? tab[idx] : __builtin_bit_cast(unsigned short, to_bf(gelu(to_f(zh))));
    }
    return r[0] | ((unsigned)r[1] << 16);
}
// v[i] = bf16(GELU(.)) of z[i]: the table when no lane of the wave holds a value
// outside it, else each value from the table or computed
template <class Tab, int N>
__device__ __forceinline__ void gelu_bf2_n(const unsigned (&z)[N], unsigned (&v)[N], const unsigned short *tab) {
    if (__builtin_amdgcn_ballot_w64(gelu_bf2_outside<Tab>(z) != 0u) == 0) {
        gelu_bf2_table<Tab>(z, v, tab);
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = gelu_bf2_word<Tab>(z[i], tab);
    }
}

// feature channel ci at position x of sample b (zero outside [0, L))
__device__ __forceinline__ float feature(const float *__restrict__ nu, const float *__restrict__ tau, int b, int L,
                                         int ci, int x) {
    if (x < 0 || x >= L) return 0.0f;
    if (ci == 0) return (nu[(int64_t)b * 2 * L + x] - 1.0f) / FS;
    if (ci == 1) return nu[(int64_t)b * 2 * L + L + x] / FS;
    return (tau[b] - TAU_C) / FS;
}

// ---------------------------------------------------------------------------
// layer 1: 3 -> 64, dilation 1, on the matrix cores.  A 16 x 16 block (16
// channels x 16 positions) is one v_mfma_f32_16x16x32_bf16 over 32 slots
// k = 8 g + j (g = lane / 16).  The features F of slot j are
//   g = 0, 1: n(t), t = 0..4, then u(0), u(1), u(2);
//   g = 2, 3: u(3), u(4), the bias slot, tau(t), t = 0..4,
// where n(t), u(t), tau(t) are the scaled n, u, tau at position x + t - 2 (zero
// outside the sample).  Even g hold bf16(F), odd g bf16(F - bf16(F)); both
// multiply the same bfloat16 weight, so each product sees about 16 bits of the
// float32 feature (the weights are bfloat16 already).  The bias slot is split
// the other way: its feature is 1 in both and its weights are the float32 bias
// as bf16(b) (g = 2) and bf16(b - bf16(b)) (g = 3).  The sum starts from zero.
// A lane's results are the 4 consecutive channels 4 g + r of position lane % 16.
// The fused inference builds the same operands, so its layer 1 equals this
// kernel's bit for bit.
// ---------------------------------------------------------------------------
constexpr int P1F = 256;
constexpr int RS = CH + 8;  // LDS row stride of a 64-channel activation row, in elements (144 bytes)
// feature slots of a lane group: (feature channel, tap) with channel 3 = the bias slot
__device__ __forceinline__ int l1_slot_ch(int s, int j) { return s == 0 ? (j < 5 ? 0 : 1) : (j < 2 ? 1 : (j == 2 ? 3 : 2)); }
__device__ __forceinline__ int l1_slot_tap(int s, int j) { return s == 0 ? (j < 5 ? j : j - 5) : (j < 2 ? 3 + j : (j == 2 ? 0 : j - 3)); }

// bf16(a), bf16(b) packed (lo = false) or the bfloat16 roundings of their
// remainders a - bf16(a), b - bf16(b) (lo = true)
__device__ __forceinline__ unsigned hl_pair(float a, float b, bool lo) {
    const unsigned hi = pack_bf2(a, b);
    const float ha = __builtin_bit_cast(float, hi << 16), hb = __builtin_bit_cast(float, hi & 0xffff0000u);
    const unsigned rem = pack_bf2(a - ha, b - hb);
    return lo ? rem : hi;
}
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
// The weight operand of channel ch for lane group g.
__device__ __forceinline__ bf16x8 l1_weights(const __bf16 *__restrict__ W1, const float *__restrict__ b1, int ch,
                                             int g) {
    auto w = [&](int t, int f) { return W1[(t * CH + ch) * 3 + f]; };
    const float bias = b1[ch];
    const __bf16 bh = to_bf(bias), bl = to_bf(bias - to_f(bh));
    if (g < 2) return bf16x8{w(0, 0), w(1, 0), w(2, 0), w(3, 0), w(4, 0), w(0, 1), w(1, 1), w(2, 1)};
    return bf16x8{w(3, 1), w(4, 1), g == 2 ? bh : bl, w(0, 2), w(1, 2), w(2, 2), w(3, 2), w(4, 2)};
}
// The features operand of a lane of group g from its 8 slot features (the bias
// slot's value is ignored).
__device__ __forceinline__ bf16x8 l1_features(const float (&F)[8], int g) {
    const bool lo = g & 1;
    u32x4_t v;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = hl_pair(F[2 * i], F[2 * i + 1], lo);
    if (g >= 2) v[1] = (v[1] & 0xffff0000u) | 0x3f80u;  // the bias slot: 1.0
    return __builtin_bit_cast(bf16x8, v);
}

// A workgroup (4 wavefronts) takes 256 positions of one sample, a wavefront 64
// (four 16-position groups, each for the 64 channels as four 16 x 16 blocks);
// the scaled n, u, tau of the workgroup's positions (with a 2-position halo) are
// staged in LDS.  A wavefront's results go through an LDS tile of its 64 rows and
// leave as 16-byte row stores: z1 (only when not null: a forward that is
// followed by a backward), then a1 = bf16(GELU(z)) by the table.
__global__ void __launch_bounds__(256) k_l1_fwd(const float *__restrict__ nu, const float *__restrict__ tau,
                                                const __bf16 *__restrict__ W1, const float *__restrict__ b1,
                                                __bf16 *__restrict__ z1, __bf16 *__restrict__ a1, int L) {
    __shared__ float fs[3][P1F + 4];
    __shared__ __attribute__((aligned(16))) __bf16 tile[4][64 * RS];  // per wavefront: 64 rows of 64 channels
    __shared__ unsigned short gt[GeluT16::N];
    const int b = blockIdx.y, x0 = blockIdx.x * P1F;
    for (int i = threadIdx.x; i < 3 * (P1F + 4); i += blockDim.x) {
        const int c = i / (P1F + 4), k = i % (P1F + 4);
        fs[c][k] = feature(nu, tau, b, L, c, x0 - 2 + k);
    }
    for (int i = threadIdx.x; i < GeluT16::N; i += blockDim.x) gt[i] = GeluT16::entry(i);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lc = lane & 15, g = lane >> 4, s = g >> 1;
    bf16x8 wa[4];
#pragma unroll
    for (int cg = 0; cg < 4; ++cg) wa[cg] = l1_weights(W1, b1, 16 * cg + lc, g);
    __syncthreads();
    __bf16 *tw = tile[wave];
    const int xw = x0 + 64 * wave;  // L is a multiple of 128: a wavefront's 64 positions are all inside or all past the end
    if (xw >= L) return;
#pragma unroll
    for (int pg = 0; pg < 4; ++pg) {
        const int xl = 64 * wave + 16 * pg;
        float F[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = l1_slot_ch(s, j);
            const float v = fs[c == 3 ? 0 : c][xl + lc + l1_slot_tap(s, j)];
            F[j] = c == 3 ? 1.0f : v;
        }
        const bf16x8 f = l1_features(F, g);
        __bf16 *trow = tw + (16 * pg + lc) * RS + 4 * g;
#pragma unroll
        for (int cg = 0; cg < 4; ++cg) {
            const floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[cg], f, floatx4{}, 0, 0, 0);
            *reinterpret_cast<uint2 *>(trow + 16 * cg) =
                make_uint2(pack_bf2(acc[0], acc[1]), pack_bf2(acc[2], acc[3]));
        }
    }
    // the wavefront's z tile, rows of 128 bytes: 8 lanes per row, 8 rows per pass
    const int rr = lane >> 3, cv = 8 * (lane & 7);
    const int64_t obase = ((int64_t)b * L + xw) * CH;
    // the tile is the wavefront's own: order its writes before the reads below
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
    for (int pass = 0; pass < 8; ++pass) {
        const int r = 8 * pass + rr;
        const bf16x8 zv = *reinterpret_cast<const bf16x8 *>(tw + r * RS + cv);
        if (z1) *reinterpret_cast<bf16x8 *>(z1 + obase + (int64_t)r * CH + cv) = zv;
        const u32x4_t zq = __builtin_bit_cast(u32x4_t, zv);
        unsigned zz[4] = {zq[0], zq[1], zq[2], zq[3]}, av[4];
        gelu_bf2_n<GeluT16>(zz, av, gt);
        *reinterpret_cast<u32x4_t *>(a1 + obase + (int64_t)r * CH + cv) = u32x4_t{av[0], av[1], av[2], av[3]};
    }
}

// ---------------------------------------------------------------------------
// 64 -> 64 layers on the matrix cores.
//   forward (DGRAD = false): out[x, n] = bias[n] + sum_{tap,k} in[x + (tap-2)d, k] Wop[tap][n][k];
//     stores a = bf16(GELU(z)) with z = bf16(out), and z itself when out_z is not null.
//   data gradient (DGRAD = true): out[x, n] = sum_{tap,k} in[x - (tap-2)d, k] Wop[tap][n][k]
//     with in = dz of the layer above and Wop the transposed weights; stores
//     dz_prev = bf16(out * GELU'(zprev[x, n])) into out_z.
// A workgroup keeps the layer's weights in LDS and walks tiles of TM = 128
// positions (b, x0) with stride gridDim.x; each of its 4 wavefronts computes 32
// positions x 64 channels as two 32 x 32 blocks (v_mfma_f32_32x32x16_bf16, K =
// 5 taps x 64 channels).  LDS rows are padded to 72 elements so that the 16-byte
// operand reads of 8 consecutive rows fall in distinct banks.  Results go back
// through LDS and leave as 16-byte row stores.
// ---------------------------------------------------------------------------
constexpr int TM = 128;
constexpr int RSF = CH + 4;  // row stride of the float32 results of the data gradient (272 bytes)

template <bool DGRAD>
__global__ void __launch_bounds__(256) k_hidden(const __bf16 *__restrict__ in, const __bf16 *__restrict__ Wop,
                                                const float *__restrict__ bias, const __bf16 *__restrict__ zprev,
                                                __bf16 *__restrict__ out_z, __bf16 *__restrict__ out_a, int B, int L,
                                                int d) {
    extern __shared__ unsigned char smem[];
    __bf16 *wl = reinterpret_cast<__bf16 *>(smem);  // [5 * 64][RS]
    __bf16 *tile = wl + KT * CH * RS;  // [TM + 4d][RS] input rows, then the results ([TM][RS] bf16 or [TM][RSF] float)
    for (int i = threadIdx.x; i < KT * CH * (CH / 8); i += blockDim.x)
        *(bf16x8 *)(wl + (i >> 3) * RS + 8 * (i & 7)) = ((const bf16x8 *)Wop)[i];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = 32 * wave, lr = lane & 31, lk = 8 * (lane >> 5);
    const int tiles_per_sample = L / TM, ntiles = B * tiles_per_sample;
    const int rows = TM + 4 * d;
    const bf16x8 zero8 = {};
    // The input rows of a tile (at most (TM + 36) x 8 vectors of 16 bytes, i.e. 6
    // per thread) are fetched into registers one tile ahead, so that their
    // latency overlaps the previous tile's matrix and epilogue work.
    constexpr int PF = ((TM + 4 * 9) * (CH / 8) + 255) / 256;
    bf16x8 pf[PF];
    auto fetch = [&](int t) {
        const int b = t / tiles_per_sample, x0 = (t % tiles_per_sample) * TM;
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int i = threadIdx.x + 256 * k;
            const int r = i >> 3, v = i & 7;
            const int pos = x0 - 2 * d + r;
            pf[k] = (r < rows && pos >= 0 && pos < L) ? *(const bf16x8 *)(in + ((int64_t)b * L + pos) * CH + 8 * v)
                                                     : zero8;
        }
    };
    if ((int)blockIdx.x < ntiles) fetch(blockIdx.x);
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int b = t / tiles_per_sample, x0 = (t % tiles_per_sample) * TM;
        __syncthreads();  // weights loaded / previous tile's results written out
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int i = threadIdx.x + 256 * k;
            if ((i >> 3) < rows) *(bf16x8 *)(tile + (i >> 3) * RS + 8 * (i & 7)) = pf[k];
        }
        __syncthreads();
        if (t + (int)gridDim.x < ntiles) fetch(t + gridDim.x);
        floatx16 acc0 = {}, acc1 = {};
        if (!DGRAD) {  // the forward sums start from the bias
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc0[r] = bias[lr];
                acc1[r] = bias[32 + lr];
            }
        }
#pragma unroll
        for (int tap = 0; tap < KT; ++tap) {
            const int off = (DGRAD ? (KT - 1 - tap) : tap) * d;
            const __bf16 *arow = tile + (m0 + lr + off) * RS + lk;
            const __bf16 *b0row = wl + (tap * CH + lr) * RS + lk;
            const __bf16 *b1row = b0row + 32 * RS;
#pragma unroll
            for (int kc = 0; kc < CH; kc += 16) {
                const bf16x8 av = *(const bf16x8 *)(arow + kc);
                const bf16x8 bv0 = *(const bf16x8 *)(b0row + kc);
                const bf16x8 bv1 = *(const bf16x8 *)(b1row + kc);
                acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv0, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv1, acc1, 0, 0, 0);
            }
        }
        __syncthreads();  // every wavefront is done reading the input tile
        // D[i][j]: i = 8 (r / 4) + 4 (lane / 32) + r % 4 (position), j = lane % 32 (channel)
        if (!DGRAD) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int pl = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                tile[pl * RS + lr] = to_bf(acc0[r]);
                tile[pl * RS + 32 + lr] = to_bf(acc1[r]);
            }
        } else {
            // float32 results (row stride 68 floats) so that GELU'(zprev) is applied
            // before the one rounding, with zprev read as whole rows below
            float *res = reinterpret_cast<float *>(tile);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int pl = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                res[pl * RSF + lr] = acc0[r];
                res[pl * RSF + 32 + lr] = acc1[r];
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < TM * (CH / 8); i += blockDim.x) {
            const int p = i >> 3, v = i & 7;
            const int64_t row = ((int64_t)b * L + x0 + p) * CH + 8 * v;
            if (!DGRAD) {
                const bf16x8 zv = *(const bf16x8 *)(tile + p * RS + 8 * v);
                if (out_z) *(bf16x8 *)(out_z + row) = zv;
                bf16x8 av;
#pragma unroll
                for (int j = 0; j < 8; ++j) av[j] = to_bf(gelu(to_f(zv[j])));
                *(bf16x8 *)(out_a + row) = av;
            } else {
                const float *res = reinterpret_cast<const float *>(tile) + p * RSF + 8 * v;
                const bf16x8 zp = *(const bf16x8 *)(zprev + row);
                bf16x8 dv;
#pragma unroll
                for (int j = 0; j < 8; ++j) dv[j] = to_bf(res[j] * gelu_grad(to_f(zp[j])));
                *(bf16x8 *)(out_z + row) = dv;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient of a 64 -> 64 layer on the matrix cores:
//   dW[tap][co][ci] = sum_{b, x} dz[b, x, co] a[b, x + (tap-2) D, ci],  db[co] = sum dz[b, x, co].
// Workgroup g takes samples g, g + G, ...; chunks of TW positions are staged in
// LDS channel-major (each lane's 8 consecutive positions contiguous).  Staging
// lanes take consecutive positions of one 8-channel group, so the transposing
// 2-byte stores of a wave land in consecutive LDS words.  The shifted operand
// a[x + (tap-2) D] starts at an odd element for odd tap * D; a second copy of
// the a tile shifted by one element keeps every operand read 4-byte aligned.
// Output: float32 partials part[g][5][64][64] and partb[g][64].
// ---------------------------------------------------------------------------
constexpr int TW = 128;

template <int D>
struct WgradTile {
    static constexpr int W = TW + 4 * D;  // staged positions of a
    static constexpr int WS = W + 2;      // row stride of the a copies (even)
    static constexpr size_t lds = (size_t)(CH * TW + 2 * CH * WS) * sizeof(__bf16);
};

__device__ __forceinline__ bf16x8 lds_read8_aligned4(const __bf16 *p) {
    const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
    typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
    u32x4 v = {q[0], q[1], q[2], q[3]};
    return __builtin_bit_cast(bf16x8, v);
}

template <int D>
__global__ void __launch_bounds__(256) k_hidden_wgrad(const __bf16 *__restrict__ dz, const __bf16 *__restrict__ a,
                                                      float *__restrict__ part, float *__restrict__ partb, int B,
                                                      int L) {
    constexpr int W = WgradTile<D>::W, WS = WgradTile<D>::WS;
    extern __shared__ unsigned char smem[];
    __bf16 *dzT = reinterpret_cast<__bf16 *>(smem);  // [64][TW]
    __bf16 *aT0 = dzT + CH * TW;                      // [64][WS]: aT0[c][p] = a[x0 - 2D + p, c]
    __bf16 *aT1 = aT0 + CH * WS;                      // [64][WS]: aT1[c][p] = aT0[c][p + 1]
    __shared__ float bred[4][CH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = 32 * (wave & 1), n0 = 32 * (wave >> 1);  // co block, ci block
    const int lr = lane & 31, lk = 8 * (lane >> 5);
    floatx16 acc[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) acc[t] = floatx16{};
    float bsum = 0.0f;
    const bf16x8 zero8 = {};
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
        for (int x0 = 0; x0 < L; x0 += TW) {
            __syncthreads();
            for (int i = threadIdx.x; i < TW * (CH / 8); i += blockDim.x) {
                const int p = i % TW, v = i / TW;
                const bf16x8 val = *(const bf16x8 *)(dz + ((int64_t)b * L + x0 + p) * CH + 8 * v);
#pragma unroll
                for (int j = 0; j < 8; ++j) dzT[(8 * v + j) * TW + p] = val[j];
            }
            for (int i = threadIdx.x; i < W * (CH / 8); i += blockDim.x) {
                const int p = i % W, v = i / W;
                const int pos = x0 - 2 * D + p;
                const bf16x8 val =
                    (pos >= 0 && pos < L) ? *(const bf16x8 *)(a + ((int64_t)b * L + pos) * CH + 8 * v) : zero8;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    aT0[(8 * v + j) * WS + p] = val[j];
                    if (p > 0) aT1[(8 * v + j) * WS + p - 1] = val[j];
                }
            }
            // bias gradient straight from global memory (rows of 64 channels, coalesced)
#pragma unroll 4
            for (int k = wave; k < TW; k += 4) bsum += to_f(dz[((int64_t)b * L + x0 + k) * CH + lane]);
            __syncthreads();
#pragma unroll 1
            for (int ks = 0; ks < TW; ks += 16) {
                const bf16x8 av = *(const bf16x8 *)(dzT + (m0 + lr) * TW + ks + lk);
#pragma unroll
                for (int tap = 0; tap < KT; ++tap) {
                    const int o = ks + lk + tap * D;
                    const bf16x8 bv = ((tap * D) & 1) ? lds_read8_aligned4(aT1 + (n0 + lr) * WS + o - 1)
                                                      : lds_read8_aligned4(aT0 + (n0 + lr) * WS + o);
                    acc[tap] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[tap], 0, 0, 0);
                }
            }
        }
    }
    float *pg = part + (int64_t)blockIdx.x * KT * CH * CH;
#pragma unroll
    for (int tap = 0; tap < KT; ++tap)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int co = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            pg[(tap * CH + co) * CH + n0 + lr] = acc[tap][r];
        }
    // bias partial: per channel (lane), the four waves' sums in a fixed order
    bred[wave][lane] = bsum;
    __syncthreads();
    if (wave == 0)
        partb[(int64_t)blockIdx.x * CH + lane] = ((bred[0][lane] + bred[1][lane]) + bred[2][lane]) + bred[3][lane];
}

// ---------------------------------------------------------------------------
// layer 4: 64 -> 2, dilation 27, on the matrix cores.  A workgroup stages the a3
// rows of its 256 positions and their +-54 halo in LDS once; then, for 16 positions at a time
// a wavefront forms y[x, c] = sum_{tap, ci} a3[x + (tap-2) 27, ci] W4[tap][c][ci] as a
// [16 x 320] x [320 x 16] product, 10 steps of v_mfma_f32_16x16x32_bf16 (K = one
// tap x 32 channels per step), the two output columns padded to 16 with zero
// weights.  A operand: lane l holds position l % 16 and channels 8 (l / 16) ..
// + 7 of the step's 32 (one 16-byte load of the a3 row); B operand: lane l holds
// column l % 16, the same 8 channels; D: lane l holds column l % 16 of
// positions 4 (l / 16) .. + 3.  Forward writes n' = n + 0.25 (b4[0] + y0) and
// u' = u + 0.25 (b4[1] + y1) ([B][2][L]).
// ---------------------------------------------------------------------------
constexpr int P4F = 256;     // positions per workgroup (4 wavefronts x 4 passes of 16)
constexpr int RS4 = CH + 8;  // LDS row stride (elements) of the staged a3 rows

__global__ void __launch_bounds__(256) k_l4_fwd(const __bf16 *__restrict__ a3, const __bf16 *__restrict__ W4,
                                                const float *__restrict__ b4, const float *__restrict__ nu,
                                                float *__restrict__ out, int L) {
    // a3 rows x0 - 54 .. x0 + 256 + 53 (zero outside [0, L)), rows padded to 72 elements
    __shared__ __bf16 rows[(P4F + 4 * 27) * RS4];
    const int b = blockIdx.y, x0 = blockIdx.x * P4F;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const bf16x8 zero8 = {};
    for (int i = threadIdx.x; i < (P4F + 4 * 27) * (CH / 8); i += blockDim.x) {
        const int r = i >> 3, v = i & 7;
        const int pos = x0 - 2 * 27 + r;
        *(bf16x8 *)(rows + r * RS4 + 8 * v) =
            (pos >= 0 && pos < L) ? *(const bf16x8 *)(a3 + ((int64_t)b * L + pos) * CH + 8 * v) : zero8;
    }
    bf16x8 bw[2 * KT];
#pragma unroll
    for (int kb = 0; kb < 2 * KT; ++kb) {
        const int tap = kb >> 1, ci = 32 * (kb & 1) + 8 * kq;
        bw[kb] = col < 2 ? *(const bf16x8 *)(W4 + (tap * 2 + col) * CH + ci) : zero8;
    }
    const float bias = col < 2 ? b4[col] : 0.0f;
    __syncthreads();
    for (int p = 16 * wave; p < P4F; p += 64) {
        if (x0 + p >= L) break;  // uniform per wavefront (L is a multiple of 128)
        floatx4 acc = {};
#pragma unroll
        for (int kb = 0; kb < 2 * KT; ++kb) {
            const int r = p + col + (kb >> 1) * 27;  // row of position x0 + p + col + (tap - 2) 27
            const bf16x8 av = *(const bf16x8 *)(rows + r * RS4 + 32 * (kb & 1) + 8 * kq);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bw[kb], acc, 0, 0, 0);
        }
        if (col < 2) {
            const int64_t o = (int64_t)b * 2 * L + (int64_t)col * L;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int xi = x0 + p + 4 * kq + r;
                out[o + xi] = nu[o + xi] + FS * (bias + acc[r]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Inference forward, all four layers in one kernel: the activations never leave
// LDS.  One workgroup (8 wavefronts) streams NS samples (one or two) from left to
// right in chunks of FC = 64 positions: sample k occupies the stream positions
// [k (L + FC), k (L + FC) + L), and the chunk between two samples is padding
// (wider than the 54-position reach of the widest layer, so no tap sees the
// other sample).  Each of a1, a2, a3 lives in a ring of FR = 256 rows (stream
// position X in row X mod 256, rows of 72 elements as above).  In iteration c,
// layer k produces the chunk of positions [64 c - D_k, 64 c - D_k + 64) with
// D = 0, 96, 192, 320: each layer lags the one below by at least a chunk plus
// its receptive half-width (2 d), so that everything it reads was written in an
// earlier iteration, and the rows a layer writes in an iteration are never read
// in that iteration (ring spans 166, 178 and 246 rows < 256).  One barrier per
// iteration.  Rows at positions outside the samples hold zeros (the zero
// padding); chunks and blocks outside skip their arithmetic (L is a multiple of
// 64, so every chunk and 32- or 16-row block lies wholly inside a sample or
// wholly outside).
// Work split: every wave takes two 16 x 16 blocks of layer 1 (operands as in
// k_l1_fwd); waves 0-3 the four 32 x 32 blocks of layer 2 and, 16 positions
// each, layer 4; waves 4-7 the blocks of layer 3.  A 32 x 32 block is channels x
// positions, with the weights as the first operand, so that a lane's results
// are 4 x 4 consecutive channels of one position (four 8-byte stores); each
// wave keeps its slices of its layers' weights in registers.  The raw n, u of the
// samples are staged in LDS before the loop (8 L bytes per sample, so
// NS L <= FMAXL), which leaves no global load inside it: a load there would make
// the wait for it also wait for the output stores in flight.  The features of
// the next chunk are written to a double buffer during each iteration.  The GELU
// is the 16 KB table (GeluT32), its reads issued together and the results
// stored; the rare wavefront with a value outside the table then replaces those
// words (a test before the reads, with the branch between them and the stores,
// cost about 4 %).  Every output element takes
// the same operations in the same order as in k_l1_fwd, k_hidden and k_l4_fwd,
// so the result equals theirs bit for bit.
// ---------------------------------------------------------------------------
constexpr int FC = 64, FR = 256, FMAXL = 4096;
constexpr int FFP = FC + 8;  // feature buffer row: positions 64 c - 2 .. 64 c + 65
// lag of layer k >= lag of layer k - 1 + one chunk + the half-width 2 d_k of its
// taps, rounded up to a multiple of 32 so that no 32-row block wraps its ring
constexpr int FD2 = 96, FD3 = 192, FD4 = 320;
static_assert(FD2 >= FC + 2 * 3 && FD3 >= FD2 + FC + 2 * 9 && FD4 >= FD3 + FC + 2 * 27, "lags cover the taps");
static_assert(FD2 % 32 == 0 && FD3 % 32 == 0 && FD4 % 32 == 0, "blocks aligned to 32 rows");
// ring span: from the lowest row read to the highest row written in one iteration
static_assert(FD2 + 2 * 3 + FC <= FR && FD3 + 2 * 9 - FD2 + FC <= FR && FD4 + 2 * 27 - FD3 + FC <= FR,
              "ring spans");
static_assert(FC >= 2 * 27, "the padding chunk between two samples covers the widest reach");
constexpr int FMAXS = 2;  // samples per workgroup (the sample of a stream position is one comparison)
constexpr size_t FUSED_RINGS = (size_t)3 * FR * RS * sizeof(__bf16);  // then NS x 2 x (L + 4) floats of n, u

__global__ void __launch_bounds__(512) k_fwd_fused(const float *__restrict__ nu, const float *__restrict__ tau,
                                                   const __bf16 *__restrict__ W1, const float *__restrict__ b1,
                                                   const __bf16 *__restrict__ W2, const float *__restrict__ b2,
                                                   const __bf16 *__restrict__ W3, const float *__restrict__ b3,
                                                   const __bf16 *__restrict__ W4, const float *__restrict__ b4,
                                                   float *__restrict__ out, int B, int L, int spw) {
    extern __shared__ unsigned char smem[];
    __bf16 *r1 = reinterpret_cast<__bf16 *>(smem);  // a1 ring [FR][RS]
    __bf16 *r2 = r1 + FR * RS;                      // a2 ring
    __bf16 *r3 = r2 + FR * RS;                      // a3 ring
    // per sample raw n then u, each with two cells of padding per side (n = 1, u = 0: features 0)
    float *nus = reinterpret_cast<float *>(smem + FUSED_RINGS);
    const int LP = L + 4;
    __shared__ unsigned short gt[GeluT32::N];       // GELU table
    __shared__ float feat[2 * 3 * FFP];             // features of the current and the next chunk
    const int s0 = blockIdx.x * spw;
    const int ns = B - s0 < spw ? B - s0 : spw;     // samples of this workgroup
    const int SL = L + FC;                          // stream stride of a sample
    const int LT = ns * SL - FC;                    // stream length
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bf16x8 zero8 = {};
    for (int i = threadIdx.x; i < 3 * FR * RS / 8; i += blockDim.x) reinterpret_cast<bf16x8 *>(smem)[i] = zero8;
    for (int i = threadIdx.x; i < GeluT32::N; i += blockDim.x) gt[i] = GeluT32::entry(i);
    for (int i = threadIdx.x; i < ns * 2 * LP; i += blockDim.x) {
        const int k = i / (2 * LP), r = i - k * 2 * LP;
        const int ch = r >= LP, x = r - ch * LP - 2;
        nus[i] = (x >= 0 && x < L) ? nu[(int64_t)(s0 + k) * 2 * L + (int64_t)ch * L + x] : (ch ? 0.0f : 1.0f);
    }
    // stream position X < 2 SL: sample k = (X >= SL), local position X - k SL
    auto inside = [&](int X) { return X >= 0 && X < LT && X - (X >= SL ? SL : 0) < L; };
    // layers 1-3: this wave's block (positions 32 mb .., channels 32 nb ..)
    const bool upper = wave >= 4;  // layer 3 and layer 1
    const int mb = wave & 1, nb = (wave >> 1) & 1;
    const int lr = lane & 31, lk = 8 * (lane >> 5);
    // layer 1: 16 positions 16 (wave % 4) .. of each chunk, channels 32 (wave / 4) ..
    // as two 16 x 16 blocks; lane = (position lc, slot group g1)
    const int lc = lane & 15, g1 = lane >> 4, s1 = g1 >> 1, pg1 = wave & 3, h1 = wave >> 2;
    bf16x8 wa1[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) wa1[q] = l1_weights(W1, b1, 32 * h1 + 16 * q + lc, g1);
    const __bf16 *Wl = upper ? W3 : W2;
    bf16x8 wb[KT][4];
#pragma unroll
    for (int tap = 0; tap < KT; ++tap)
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
            wb[tap][kc] = *(const bf16x8 *)(Wl + (int64_t)(tap * CH + nb * 32 + lr) * CH + 16 * kc + lk);
    // layer 4 (waves 0-3): lane = (position col within 16, channel quarter kq)
    const int col = lane & 15, kq = lane >> 4;
    bf16x8 bw[2 * KT];
#pragma unroll
    for (int kb = 0; kb < 2 * KT; ++kb) {
        const int tap = kb >> 1, ci = 32 * (kb & 1) + 8 * kq;
        bw[kb] = col < 2 ? *(const bf16x8 *)(W4 + (tap * 2 + col) * CH + ci) : zero8;
    }
    const float bias4 = col < 2 ? b4[col] : 0.0f;
    // layers 2 / 3: the biases of this lane's 16 result channels
    // nb 32 + 8 (r / 4) + 4 (lane / 32) + r % 4
    floatx16 bz;
#pragma unroll
    for (int r = 0; r < 16; ++r) bz[r] = (upper ? b3 : b2)[nb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)];
    // per sample: the tau feature
    float ftau[FMAXS];
#pragma unroll
    for (int k = 0; k < FMAXS; ++k) ftau[k] = k < ns ? (tau[s0 + k] - TAU_C) / FS : 0.0f;
    const int d = upper ? 9 : 3, D = upper ? FD3 : FD2;
    const __bf16 *rin = upper ? r2 : r1;
    __bf16 *rout = upper ? r3 : r2;
    const int niter = (LT + FD4 - 1) / FC + 1;
    // Let the weight loads land before the loop: otherwise the compiler's wait
    // counts inside the loop stay conservative and every iteration's last matrix
    // operation waits for all vector-memory traffic in flight (the previous
    // chunk's stores).  vmcnt(0), the other counters free.
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();

    // layer 1: two 16 x 16 blocks (operands as in k_l1_fwd)
    auto layer1 = [&](int c) {
        const int X = c * FC + 16 * pg1 + lc;  // this lane's position
        __bf16 *orow = r1 + (X & (FR - 1)) * RS + 32 * h1 + 4 * g1;
        if (!inside(c * FC)) {
#pragma unroll
            for (int q = 0; q < 2; ++q) *reinterpret_cast<uint2 *>(orow + 16 * q) = make_uint2(0u, 0u);
        } else {
            const float *fb = feat + (c & 1) * 3 * FFP + 16 * pg1 + lc;
            float F[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int ch = l1_slot_ch(s1, j);
                const float v = fb[(ch == 3 ? 0 : ch) * FFP + l1_slot_tap(s1, j)];
                F[j] = ch == 3 ? 1.0f : v;
            }
            const bf16x8 f = l1_features(F, g1);
            unsigned zq[4], g[4];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa1[q], f, floatx4{}, 0, 0, 0);
                zq[2 * q] = pack_bf2(acc[0], acc[1]);
                zq[2 * q + 1] = pack_bf2(acc[2], acc[3]);
            }
            gelu_bf2_table<GeluT32>(zq, g, gt);
#pragma unroll
            for (int q = 0; q < 2; ++q) *reinterpret_cast<uint2 *>(orow + 16 * q) = make_uint2(g[2 * q], g[2 * q + 1]);
            if (__builtin_amdgcn_ballot_w64(gelu_bf2_outside<GeluT32>(zq) != 0u) != 0) {  // rare
#pragma unroll
                for (int i = 0; i < 4; ++i) g[i] = gelu_bf2_word<GeluT32>(zq[i], gt);
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    *reinterpret_cast<uint2 *>(orow + 16 * q) = make_uint2(g[2 * q], g[2 * q + 1]);
            }
        }
    };
    // layer 2 (waves 0-3) or 3 (waves 4-7): one 32 x 32 block, channels x positions
    auto block = [&](int c) {
        const int p0 = c * FC - D + 32 * mb;  // a multiple of 32: the block's rows do not wrap
        // result element r of this lane: position p0 + lr, channel nb 32 + 8 (r / 4) + 4 (lane / 32) + r % 4
        __bf16 *orow = rout + ((p0 + lr) & (FR - 1)) * RS + nb * 32 + 4 * (lane >> 5);
        if (!inside(p0)) {
#pragma unroll
            for (int q = 0; q < 4; ++q) *reinterpret_cast<uint2 *>(orow + 8 * q) = make_uint2(0u, 0u);
        } else {
            floatx16 acc = bz;  // the sums start from the bias
            // the operands of tap t + 1 are read while tap t's products run (the
            // scheduling barriers keep the compiler from moving the reads back
            // next to their products, where each pair waited for its own reads)
            bf16x8 av[2][4];
            auto fetch = [&](int tap, bf16x8 (&v)[4]) {
                const __bf16 *arow = rin + ((p0 + lr + (tap - 2) * d) & (FR - 1)) * RS + lk;
#pragma unroll
                for (int kc = 0; kc < 4; ++kc) v[kc] = *(const bf16x8 *)(arow + 16 * kc);
            };
            fetch(0, av[0]);
#pragma unroll
            for (int tap = 0; tap < KT; ++tap) {
                if (tap + 1 < KT) fetch(tap + 1, av[(tap + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int kc = 0; kc < 4; ++kc)
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wb[tap][kc], av[tap & 1][kc], acc, 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
            unsigned zq[8], g[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) zq[i] = pack_bf2(acc[2 * i], acc[2 * i + 1]);
            gelu_bf2_table<GeluT32>(zq, g, gt);
#pragma unroll
            for (int q = 0; q < 4; ++q) *reinterpret_cast<uint2 *>(orow + 8 * q) = make_uint2(g[2 * q], g[2 * q + 1]);
            if (__builtin_amdgcn_ballot_w64(gelu_bf2_outside<GeluT32>(zq) != 0u) != 0) {  // rare
#pragma unroll
                for (int i = 0; i < 8; ++i) g[i] = gelu_bf2_word<GeluT32>(zq[i], gt);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    *reinterpret_cast<uint2 *>(orow + 8 * q) = make_uint2(g[2 * q], g[2 * q + 1]);
            }
        }
    };
    // layer 4 (waves 0-3): 16 positions each, n' = n + 0.25 (b4 + y)
    auto layer4 = [&](int c) {
        const int p = c * FC - FD4 + 16 * wave;
        if (inside(p)) {
            floatx4 acc = {};
            bf16x8 av[2 * KT];  // all ten operands read before the first product
#pragma unroll
            for (int kb = 0; kb < 2 * KT; ++kb) {
                const int pos = p + col + ((kb >> 1) - 2) * 27;
                av[kb] = *(const bf16x8 *)(r3 + (pos & (FR - 1)) * RS + 32 * (kb & 1) + 8 * kq);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int kb = 0; kb < 2 * KT; ++kb)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[kb], bw[kb], acc, 0, 0, 0);
            if (col < 2) {
                const int k = p >= SL, xl = p - k * SL;
                const int64_t o = (int64_t)(s0 + k) * 2 * L + (int64_t)col * L;
                const float *nk = nus + k * 2 * LP + col * LP + 2;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int xi = xl + 4 * kq + r;
                    out[o + xi] = nk[xi] + FS * (bias4 + acc[r]);
                }
            }
        }
    };
    // the features n, u, tau of stream positions 64 (c + 1) - 2 .. 64 (c + 1) + 65
    // into the feature buffer of chunk c + 1 (zero outside the samples), by the
    // first 204 threads
    auto features = [&](int c) {
        const int i = threadIdx.x;
        if (i < 3 * (FC + 4)) {
            const int ch = i / (FC + 4), q = i % (FC + 4);
            const int X = (c + 1) * FC - 2 + q;
            float v = 0.0f;
            if (inside(X)) {
                const int k = X >= SL, xl = X - k * SL;
                if (ch == 2) {
                    v = k ? ftau[1] : ftau[0];
                } else {
                    const float raw = nus[k * 2 * LP + ch * LP + xl + 2];
                    v = ch == 0 ? (raw - 1.0f) / FS : raw / FS;
                }
            }
            feat[((c + 1) & 1) * 3 * FFP + ch * FFP + q] = v;
        }
    };
    features(-1);
    __syncthreads();
    // The sections of an iteration read only what earlier iterations wrote, so
    // their order within an iteration is free.
    for (int c = 0; c < niter; ++c) {
        layer1(c);
        block(c);
        if (!upper) layer4(c);
        features(c);
        __syncthreads();
    }
}

// Data gradient through layer 4 and the GELU of layer 3:
//   da3[x, ci] = sum_{tap, c} dy[c, x - (tap-2) 27] W4[tap][c][ci],  dz3 = bf16(da3 GELU'(z3)),
// with dy = 0.25 dout (the residual's scale).  8 threads per position, 8 channels each.
__global__ void __launch_bounds__(256) k_l4_dgrad(const float *__restrict__ dout, const __bf16 *__restrict__ W4,
                                                  const __bf16 *__restrict__ z3, __bf16 *__restrict__ dz3, int L) {
    __shared__ float w[KT * 2 * CH];
    for (int i = threadIdx.x; i < KT * 2 * CH; i += blockDim.x) w[i] = to_f(W4[i]);
    __syncthreads();
    const int b = blockIdx.y, x = blockIdx.x * 32 + (threadIdx.x >> 3), c8 = 8 * (threadIdx.x & 7);
    if (x >= L) return;
    float dyv[KT][2];
#pragma unroll
    for (int tap = 0; tap < KT; ++tap) {
        const int pos = x - (tap - 2) * 27;
        const bool ok = pos >= 0 && pos < L;
        dyv[tap][0] = ok ? FS * dout[(int64_t)b * 2 * L + pos] : 0.0f;
        dyv[tap][1] = ok ? FS * dout[(int64_t)b * 2 * L + L + pos] : 0.0f;
    }
    const int64_t row = ((int64_t)b * L + x) * CH + c8;
    const bf16x8 zv = *(const bf16x8 *)(z3 + row);
    bf16x8 dv;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int ci = c8 + j;
        float acc = 0.0f;
#pragma unroll
        for (int tap = 0; tap < KT; ++tap) {
            acc = __builtin_fmaf(dyv[tap][0], w[(tap * 2 + 0) * CH + ci], acc);
            acc = __builtin_fmaf(dyv[tap][1], w[(tap * 2 + 1) * CH + ci], acc);
        }
        dv[j] = to_bf(acc * gelu_grad(to_f(zv[j])));
    }
    *(bf16x8 *)(dz3 + row) = dv;
}

// Fixed-order sum of 256 per-thread values (tree over an LDS array).
__device__ __forceinline__ float block_sum256(float v, float *scratch) {
    scratch[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) scratch[threadIdx.x] += scratch[threadIdx.x + s];
        __syncthreads();
    }
    const float r = scratch[0];
    __syncthreads();
    return r;
}

// Weight gradient of layer 4: dW4[tap][c][ci] = sum_{b,x} dy[b, c, x] a3[b, x + (tap-2) 27, ci],
// db4[c] = sum dy.  Workgroup g takes samples g, g + G, ...; thread (ci = t % 64,
// group t / 64) walks a3 rows of chunks of 256 positions, with dy of the chunk
// (and a 54-position halo) staged in LDS.  Partials part[g][642].
constexpr int P4 = 256, H4 = 2 * 27;

__global__ void __launch_bounds__(256) k_l4_wgrad(const float *__restrict__ dout, const __bf16 *__restrict__ a3,
                                                  float *__restrict__ part, int B, int L) {
    constexpr int NW = KT * 2 * CH;
    __shared__ float dyl[2][P4 + 2 * H4];
    __shared__ float red[4][NW];
    __shared__ float tmp[256];
    const int ci = threadIdx.x & 63, grp = threadIdx.x >> 6;
    float acc[KT][2] = {};
    float bacc0 = 0.0f, bacc1 = 0.0f;
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
        const float *dyb = dout + (int64_t)b * 2 * L;
        for (int p0 = 0; p0 < L; p0 += P4) {
            __syncthreads();
            for (int i = threadIdx.x; i < 2 * (P4 + 2 * H4); i += blockDim.x) {
                const int c = i / (P4 + 2 * H4), k = i % (P4 + 2 * H4);
                const int x = p0 - H4 + k;
                dyl[c][k] = (x >= 0 && x < L) ? FS * dyb[c * L + x] : 0.0f;
            }
            __syncthreads();
            if (p0 + threadIdx.x < L) {
                bacc0 += dyl[0][H4 + threadIdx.x];
                bacc1 += dyl[1][H4 + threadIdx.x];
            }
            const int kend = min(P4, L - p0);
#pragma unroll 4
            for (int k = grp; k < kend; k += 4) {
                const float a = to_f(a3[((int64_t)b * L + p0 + k) * CH + ci]);
#pragma unroll
                for (int tap = 0; tap < KT; ++tap) {
                    const int idx = k + H4 - (tap - 2) * 27;
                    acc[tap][0] = __builtin_fmaf(dyl[0][idx], a, acc[tap][0]);
                    acc[tap][1] = __builtin_fmaf(dyl[1][idx], a, acc[tap][1]);
                }
            }
        }
    }
#pragma unroll
    for (int tap = 0; tap < KT; ++tap) {
        red[grp][(tap * 2 + 0) * CH + ci] = acc[tap][0];
        red[grp][(tap * 2 + 1) * CH + ci] = acc[tap][1];
    }
    __syncthreads();
    float *pg = part + (int64_t)blockIdx.x * (NW + 2);
    for (int o = threadIdx.x; o < NW; o += blockDim.x) pg[o] = ((red[0][o] + red[1][o]) + red[2][o]) + red[3][o];
    const float s0 = block_sum256(bacc0, tmp);
    const float s1 = block_sum256(bacc1, tmp);
    if (threadIdx.x == 0) {
        pg[NW] = s0;
        pg[NW + 1] = s1;
    }
}

// Weight gradient of layer 1: dW1[tap][co][ci] = sum_{b,x} dz1[b, x, co] f[b, ci, x + tap - 2],
// db1[co] = sum dz1.  Thread (co = t % 64, group t / 64) walks the positions of
// chunks of 256 with the chunk's features (and a 2-position halo) in LDS.
// Partials part[g][5*64*3 + 64].
constexpr int P1W = 256;

__global__ void __launch_bounds__(256) k_l1_wgrad(const __bf16 *__restrict__ dz1, const float *__restrict__ nu,
                                                  const float *__restrict__ tau, float *__restrict__ part, int B,
                                                  int L) {
    constexpr int NW = KT * CH * 3;
    __shared__ float red[4][NW + CH];
    __shared__ float fs[3][P1W + 4];
    const int co = threadIdx.x & 63, grp = threadIdx.x >> 6;
    float acc[KT][3] = {};
    float bacc = 0.0f;
    for (int b = blockIdx.x; b < B; b += gridDim.x) {
        for (int p0 = 0; p0 < L; p0 += P1W) {
            __syncthreads();
            for (int i = threadIdx.x; i < 3 * (P1W + 4); i += blockDim.x) {
                const int c = i / (P1W + 4), k = i % (P1W + 4);
                fs[c][k] = feature(nu, tau, b, L, c, p0 - 2 + k);
            }
            __syncthreads();
            const int kend = min(P1W, L - p0);
#pragma unroll 4
            for (int k = grp; k < kend; k += 4) {
                const float g = to_f(dz1[((int64_t)b * L + p0 + k) * CH + co]);
                bacc += g;
#pragma unroll
                for (int t = 0; t < KT; ++t)
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[t][c] = __builtin_fmaf(g, fs[c][k + t], acc[t][c]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < KT; ++t)
#pragma unroll
        for (int c = 0; c < 3; ++c) red[grp][(t * CH + co) * 3 + c] = acc[t][c];
    red[grp][NW + co] = bacc;
    __syncthreads();
    for (int o = threadIdx.x; o < NW + CH; o += blockDim.x)
        part[(int64_t)blockIdx.x * (NW + CH) + o] = ((red[0][o] + red[1][o]) + red[2][o]) + red[3][o];
}

// dst[i] = sum over g of part[g][i] in a fixed order: four interleaved partial
// sums (g = j mod 4), then ((s0 + s1) + s2) + s3.  64 outputs per workgroup.
__global__ void __launch_bounds__(256) k_reduce(const float *__restrict__ part, int G, int n, float *__restrict__ dst) {
    __shared__ float sums[4][64];
    const int t = threadIdx.x & 63, j = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + t;
    float a = 0.0f;
    if (i < n) {
#pragma unroll 8
        for (int g = j; g < G; g += 4) a += part[(int64_t)g * n + i];
    }
    sums[j][t] = a;
    __syncthreads();
    if (j == 0 && i < n) dst[i] = ((sums[0][t] + sums[1][t]) + sums[2][t]) + sums[3][t];
}

// ---------------------------------------------------------------------------
// loss: e = (out - target) / 0.25 over both fields; L = mean(e^2) + lambda mean_b (mean_x e0)^2
// (the second term asks for conserved mass without enforcing it).
// dout = dL/d out; per-sample sums of e^2 and e0 written to stats[b][2].
// One workgroup per sample.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_loss(const float *__restrict__ out, const float *__restrict__ target,
                                              float *__restrict__ dout, float *__restrict__ stats, int B, int L,
                                              float lambda_mass) {
    const int b = blockIdx.x;
    const int64_t o = (int64_t)b * 2 * L;
    float se = 0.0f, s0 = 0.0f;
    for (int i = threadIdx.x; i < 2 * L; i += blockDim.x) {
        const float e = (out[o + i] - target[o + i]) / FS;
        se += e * e;
        if (i < L) s0 += e;
    }
    __shared__ float r1[256], r2[256];
    r1[threadIdx.x] = se;
    r2[threadIdx.x] = s0;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
        }
        __syncthreads();
    }
    const float mean_e0 = r2[0] / L;
    const float N = float(B) * 2.0f * L;
    for (int i = threadIdx.x; i < 2 * L; i += blockDim.x) {
        const float e = (out[o + i] - target[o + i]) / FS;
        float g = 2.0f * e / N;
        if (i < L) g += lambda_mass * 2.0f * mean_e0 / (float(B) * L);
        dout[o + i] = g / FS;
    }
    if (threadIdx.x == 0) {
        stats[2 * b] = r1[0];
        stats[2 * b + 1] = mean_e0;
    }
}

// per-sample relative mass residual |sum n' - sum n| / sum n of a prediction
__global__ void __launch_bounds__(256) k_mass_residual(const float *__restrict__ in, const float *__restrict__ out,
                                                       float *__restrict__ resid, int L) {
    const int b = blockIdx.x;
    const int64_t o = (int64_t)b * 2 * L;
    double s_in = 0.0, s_out = 0.0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        s_in += in[o + i];
        s_out += out[o + i];
    }
    __shared__ double r1[256], r2[256];
    r1[threadIdx.x] = s_in;
    r2[threadIdx.x] = s_out;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) resid[b] = float(fabs(r2[0] - r1[0]) / r1[0]);
}

// Acceptance indicator of a prediction for the hybrid advance: the relative
// mass residual as above, or +inf when any predicted value is not finite or
// any predicted density is not positive (a state the lattice step cannot take).
__global__ void __launch_bounds__(256) k_indicator(const float *__restrict__ in, const float *__restrict__ out,
                                                   float *__restrict__ resid, int L) {
    const int b = blockIdx.x;
    const int64_t o = (int64_t)b * 2 * L;
    double s_in = 0.0, s_out = 0.0;
    int bad = 0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const float n1 = out[o + i], u1 = out[o + L + i];
        bad |= (int)!(n1 > 0.0f) | (int)!isfinite(n1) | (int)!isfinite(u1);
        s_in += in[o + i];
        s_out += n1;
    }
    __shared__ double r1[256], r2[256];
    __shared__ int rb[256];
    r1[threadIdx.x] = s_in;
    r2[threadIdx.x] = s_out;
    rb[threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
            rb[threadIdx.x] |= rb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) resid[b] = rb[0] ? __builtin_inff() : float(fabs(r2[0] - r1[0]) / r1[0]);
}


// ---------------------------------------------------------------------------
// Adam on the float32 master vector (bias-corrected), then the bfloat16 copies.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                                              const float *__restrict__ g, int n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 copies: plain copy for [tap][co][ci] and the transposed [tap][ci][co] of a 64x64 layer
__global__ void __launch_bounds__(256) k_to_bf16(const float *__restrict__ src, __bf16 *__restrict__ dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = to_bf(src[i]);
}

__global__ void __launch_bounds__(256) k_transpose_bf16(const float *__restrict__ src, __bf16 *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= KT * CH * CH) return;
    const int tap = i / (CH * CH), co = (i / CH) % CH, ci = i % CH;
    dst[(tap * CH + ci) * CH + co] = to_bf(src[i]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t l1_fwd(const float *nu, const float *tau, const __bf16 *W1, const float *b1, __bf16 *z1, __bf16 *a1, int B,
                  int L, hipStream_t s) {
    hipLaunchKernelGGL(k_l1_fwd, dim3((L + P1F - 1) / P1F, B), dim3(256), 0, s, nu, tau, W1, b1, z1, a1, L);
    return hipGetLastError();
}

// Kernels with more than 64 KB of dynamic LDS need their limit raised, on each
// device they run on: once per device and kernel, under a lock.
constexpr int kMaxDevices = 64;
struct LdsLimit {
    std::mutex m;
    bool done[kMaxDevices] = {};
    hipError_t raise(const void *fn, int bytes) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
        std::lock_guard<std::mutex> lock(m);
        if (done[dev]) return hipSuccess;
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e == hipSuccess) done[dev] = true;
        return e;
    }
};

size_t hidden_lds(int d, bool dgrad) {
    size_t tile = (size_t)(TM + 4 * d) * RS * sizeof(__bf16);
    if (dgrad && tile < (size_t)TM * RSF * sizeof(float)) tile = (size_t)TM * RSF * sizeof(float);
    return (size_t)KT * CH * RS * sizeof(__bf16) + tile;
}

hipError_t hidden(bool dgrad, const __bf16 *in, const __bf16 *Wop, const float *bias, const __bf16 *zprev,
                  __bf16 *out_z, __bf16 *out_a, int B, int L, int d, hipStream_t s) {
    if (L % TM) return hipErrorInvalidValue;
    static LdsLimit fwd_limit, dgrad_limit;
    hipError_t attr = dgrad ? dgrad_limit.raise((const void *)k_hidden<true>, (int)hidden_lds(9, true))
                            : fwd_limit.raise((const void *)k_hidden<false>, (int)hidden_lds(9, false));
    if (attr != hipSuccess) return attr;
    if (d != 3 && d != 9) return hipErrorInvalidValue;
    const int ntiles = B * (L / TM);
    const int grid = ntiles < 512 ? ntiles : 512;  // two workgroups per CU (about 70 KB of LDS each)
    if (dgrad)
        hipLaunchKernelGGL(k_hidden<true>, dim3(grid), dim3(256), hidden_lds(d, true), s, in, Wop, bias, zprev, out_z, out_a,
                           B, L, d);
    else
        hipLaunchKernelGGL(k_hidden<false>, dim3(grid), dim3(256), hidden_lds(d, false), s, in, Wop, bias, zprev, out_z,
                           out_a, B, L, d);
    return hipGetLastError();
}

hipError_t hidden_wgrad(const __bf16 *dz, const __bf16 *a, float *part, float *partb, int G, int B, int L, int d,
                        hipStream_t s) {
    if (d == 3)
        hipLaunchKernelGGL(k_hidden_wgrad<3>, dim3(G), dim3(256), WgradTile<3>::lds, s, dz, a, part, partb, B, L);
    else if (d == 9)
        hipLaunchKernelGGL(k_hidden_wgrad<9>, dim3(G), dim3(256), WgradTile<9>::lds, s, dz, a, part, partb, B, L);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

int fused_max_length() { return FMAXL; }

// Compute units of the current device (cached per device).
static int device_cus() {
    static std::mutex m;
    static int cus[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
    std::lock_guard<std::mutex> lock(m);
    if (cus[dev] == 0 && hipDeviceGetAttribute(&cus[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus[dev] = 0;
    return cus[dev];
}

hipError_t fwd_fused(const float *nu, const float *tau, const __bf16 *W1, const float *b1, const __bf16 *W2,
                     const float *b2, const __bf16 *W3, const float *b3, const __bf16 *W4, const float *b4, float *out,
                     int B, int L, hipStream_t s) {
    if (B < 1 || L < FC || L % FC || L > FMAXL) return hipErrorInvalidValue;
    static LdsLimit limit;
    constexpr size_t kMaxStage = (size_t)2 * (FMAXL + 4) > (size_t)FMAXS * 2 * (FMAXL / FMAXS + 4)
                                     ? (size_t)2 * (FMAXL + 4)
                                     : (size_t)FMAXS * 2 * (FMAXL / FMAXS + 4);
    // with the static LDS (the GELU table and the feature buffers), within the 160 KiB of a workgroup
    static_assert(FUSED_RINGS + kMaxStage * sizeof(float) + GeluT32::N * sizeof(unsigned short) +
                          2 * 3 * FFP * sizeof(float) <= 160 * 1024,
                  "LDS of the largest staging");
    const hipError_t attr = limit.raise((const void *)k_fwd_fused, (int)(FUSED_RINGS + kMaxStage * sizeof(float)));
    if (attr != hipSuccess) return attr;
    // two samples per workgroup once there are more samples than compute units
    // (one workgroup fits a CU): the padding chunk between them replaces the
    // pipeline's fill and drain, and no second wave of workgroups is needed
    const int cus = device_cus();
    const int spw = (cus > 0 && B > cus && L * FMAXS <= FMAXL) ? FMAXS : 1;
    const int grid = (B + spw - 1) / spw;
    const size_t lds = FUSED_RINGS + (size_t)spw * 2 * (L + 4) * sizeof(float);
    hipLaunchKernelGGL(k_fwd_fused, dim3(grid), dim3(512), lds, s, nu, tau, W1, b1, W2, b2, W3, b3, W4, b4, out, B, L,
                       spw);
    return hipGetLastError();
}

hipError_t l4_fwd(const __bf16 *a3, const __bf16 *W4, const float *b4, const float *nu, float *out, int B, int L,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_l4_fwd, dim3((L + P4F - 1) / P4F, B), dim3(256), 0, s, a3, W4, b4, nu, out, L);
    return hipGetLastError();
}

hipError_t l4_dgrad(const float *dout, const __bf16 *W4, const __bf16 *z3, __bf16 *dz3, int B, int L, hipStream_t s) {
    hipLaunchKernelGGL(k_l4_dgrad, dim3((L + 31) / 32, B), dim3(256), 0, s, dout, W4, z3, dz3, L);
    return hipGetLastError();
}

hipError_t l4_wgrad(const float *dout, const __bf16 *a3, float *part, int G, int B, int L, hipStream_t s) {
    hipLaunchKernelGGL(k_l4_wgrad, dim3(G), dim3(256), 0, s, dout, a3, part, B, L);
    return hipGetLastError();
}

hipError_t l1_wgrad(const __bf16 *dz1, const float *nu, const float *tau, float *part, int G, int B, int L,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_l1_wgrad, dim3(G), dim3(256), 0, s, dz1, nu, tau, part, B, L);
    return hipGetLastError();
}

hipError_t reduce(const float *part, int G, int n, float *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3((n + 63) / 64), dim3(256), 0, s, part, G, n, dst);
    return hipGetLastError();
}

hipError_t loss(const float *out, const float *target, float *dout, float *stats, int B, int L, float lambda,
                hipStream_t s) {
    hipLaunchKernelGGL(k_loss, dim3(B), dim3(256), 0, s, out, target, dout, stats, B, L, lambda);
    return hipGetLastError();
}

hipError_t mass_residual(const float *in, const float *out, float *resid, int B, int L, hipStream_t s) {
    hipLaunchKernelGGL(k_mass_residual, dim3(B), dim3(256), 0, s, in, out, resid, L);
    return hipGetLastError();
}

hipError_t indicator(const float *in, const float *out, float *resid, int B, int L, hipStream_t s) {
    hipLaunchKernelGGL(k_indicator, dim3(B), dim3(256), 0, s, in, out, resid, L);
    return hipGetLastError();
}

hipError_t adam(float *p, float *m, float *v, const float *g, int n, float lr, float b1, float b2, float eps, float c1,
                float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t to_bf16(const float *src, __bf16 *dst, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t transpose_bf16(const float *src, __bf16 *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose_bf16, dim3((KT * CH * CH + 255) / 256), dim3(256), 0, s, src, dst);
    return hipGetLastError();
}

}  // namespace srg
