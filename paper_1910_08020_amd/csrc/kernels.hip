// HIP kernels for the Trotterized Z2 lattice-gauge state vector on CDNA4 (gfx950).
//
// One Trotter substep (Sec. 2.2 of arXiv:1910.08020) is a link layer
// prod_l exp(i a sigma^x_l) followed by the diagonal plaquette phase
// exp(i theta sum_p U_p).  The link layer is a tensor product of identical
// 2x2 rotations, applied in a few passes over HBM:
//   * low pass: a contiguous tile of 2^12 amplitudes staged through LDS, all
//     twelve low link qubits rotated in registers between LDS transposes;
//   * high passes: each lane keeps 2^h amplitudes that differ in h higher
//     link qubits in registers, with lanes of a wave on consecutive
//     amplitudes, so every load instruction reads one contiguous segment.
// The plaquette phase is folded into the last pass: the plaquette syndrome
// P(b) (bit p = parity of plaquette p on basis state b) is linear over GF(2),
// so P(base | r) = P(base) ^ P(r) with P(base) from byte tables in LDS and
// P(r) from the per-link plaquette sets; the phase is table[popcount(P)].
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <algorithm>
#include <mutex>
#include <type_traits>

#include "lgt_internal.hpp"
#include "tile_layout.hpp"

namespace lgt {

template <typename T> struct CV;
template <> struct CV<float> { using type = float2; };
template <> struct CV<double> { using type = double2; };

template <typename T>
using cplx_t = typename CV<T>::type;

// Pointers taken from DevInst records are generic; casting them to the global address
// space makes the compiler emit global (not flat) loads and stores, which count only
// against vmcnt, so waits on LDS traffic do not also wait for prefetched tiles.
template <typename X>
using gp = __attribute__((address_space(1))) X *;
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));

// element loads and stores through global pointers (pairs as native 2-vectors)
template <typename T>
__device__ __forceinline__ cplx_t<T> ldg(gp<const cplx_t<T>> p)
{
    const vec2<T> v = *(gp<const vec2<T>>)p;
    cplx_t<T> c;
    c.x = v.x;
    c.y = v.y;
    return c;
}
__device__ __forceinline__ float2 ldg(gp<const float2> p) { return ldg<float>(p); }
__device__ __forceinline__ double2 ldg(gp<const double2> p) { return ldg<double>(p); }
template <typename T>
__device__ __forceinline__ RotParam<T> ldg(gp<const RotParam<T>> p)
{
    const vec2<T> v = *(gp<const vec2<T>>)p;
    return RotParam<T>{v.x, v.y};
}
template <typename C>
__device__ __forceinline__ void stg(gp<C> p, const C &c)
{
    using T = std::remove_reference_t<decltype(c.x)>;
    vec2<T> v;
    v.x = c.x;
    v.y = c.y;
    *(gp<vec2<T>>)p = v;
}
// the same store marked non-temporal (streaming: the data is not expected back soon)
template <typename C>
__device__ __forceinline__ void stg_nt(gp<C> p, const C &c)
{
    using T = std::remove_reference_t<decltype(c.x)>;
    vec2<T> v;
    v.x = c.x;
    v.y = c.y;
    __builtin_nontemporal_store(v, (gp<vec2<T>>)p);
}

constexpr int kPtabWords = kParityBytes * 256;

__device__ __forceinline__ uint32_t syndrome(uint64_t b, const uint32_t *tab)
{
    return tab[(uint32_t)b & 255u] ^ tab[256 + (((uint32_t)b >> 8) & 255u)] ^
           tab[512 + (((uint32_t)b >> 16) & 255u)] ^ tab[768 + (((uint32_t)b >> 24) & 255u)] ^
           tab[1024 + ((uint32_t)(b >> 32) & 255u)];
}

// plaquettes touching link q, read from the byte tables (single-bit entry)
__device__ __forceinline__ uint32_t link_set(int q, const uint32_t *tab)
{
    return tab[(q >> 3) * 256 + (1 << (q & 7))];
}

__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// a * b for a phase factor b (a table entry or an R_z gate).  Over small time steps b.x lies within a few ulps of
// +-1; a product by such a factor, rounded on its own, moves by a whole ulp or not at all,
// the same way every step, and the norm of a complex64 state drifted by 1e-8 per step.
// Here the products with b.x stay inside the FMA and are rounded once together with the
// b.y terms.
template <typename C>
__device__ __forceinline__ C cmul_ph(C a, C b)
{
    C r;
    r.x = fma_r(a.x, b.x, -(a.y * b.y));
    r.y = fma_r(a.y, b.x, a.x * b.y);
    return r;
}

// (a0, a1) <- (u a0 + i v a1, i v a0 + u a1): the link rotation up to the scale
// folded into the phase table.  One of u, v is exactly 1.
template <typename T, typename C>
__device__ __forceinline__ void rot_pair(C &a0, C &a1, T u, T v)
{
    C b0, b1;
    b0.x = u * a0.x - v * a1.y;
    b0.y = u * a0.y + v * a1.x;
    b1.x = u * a1.x - v * a0.y;
    b1.y = u * a1.y + v * a0.x;
    a0 = b0;
    a1 = b1;
}

// rotate every register bit of a 2^B register array
template <typename T, typename C, int B>
__device__ __forceinline__ void rot_regs(C *v, T u, T w)
{
#pragma unroll
    for (int k = 0; k < B; ++k)
#pragma unroll
        for (int r = 0; r < (1 << B); ++r)
            if (!(r & (1 << k))) rot_pair<T, C>(v[r], v[r | (1 << k)], u, w);
}

// multiply a 2^B register array (register r <-> global index base | sum_k r_k 2^{q_k})
// by table[popcount(P0 ^ P(r))], qs holding the plaquette sets of the register bits
template <typename C, int B>
__device__ __forceinline__ void apply_phase_regs(C *v, uint32_t P0, const uint32_t *qs,
                                                 const C *table)
{
#pragma unroll
    for (int r = 0; r < (1 << B); ++r) {
        uint32_t P = P0;
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (r & (1 << k)) P ^= qs[k];
        v[r] = cmul_ph(v[r], table[__popc(P)]);
    }
}

// multiply 16 registers by table[popcount(P0 ^ pr[r])], pr[r] the (uniform) plaquette set
// of register r's index bits
template <typename C>
__device__ __forceinline__ void apply_phase_pr(C *v, uint32_t P0, const uint32_t *pr, const C *table)
{
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = cmul_ph(v[r], table[__popc(P0 ^ pr[r])]);
}

// plaquette sets of the 16 register combinations from the 4 single-bit sets, kept in
// scalar registers (the sets are the same for every lane)
__device__ __forceinline__ void reg_sets(const uint32_t *q, uint32_t *pr)
{
    uint32_t s[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) s[k] = __builtin_amdgcn_readfirstlane(q[k]);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        uint32_t x = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (r & (1 << k)) x ^= s[k];
        pr[r] = x;
    }
}

template <typename T>
__device__ __forceinline__ void load_tables(const DevInst &in, int n_plaq, int pre, int post,
                                            uint32_t *ptab, cplx_t<T> *ph_pre,
                                            cplx_t<T> *ph_post)
{
    using C = cplx_t<T>;
    const gp<const uint32_t> gtab = (gp<const uint32_t>)in.ptab;
    for (int i = threadIdx.x; i < kPtabWords; i += blockDim.x) ptab[i] = gtab[i];
    const gp<const C> ph = (gp<const C>)in.phase;
    const int np1 = n_plaq + 1;
    if (pre >= 0)
        for (int i = threadIdx.x; i < np1; i += blockDim.x)
            ph_pre[i] = ldg(ph + (size_t)(in.ph0 + pre) * np1 + i);
    if (post >= 0)
        for (int i = threadIdx.x; i < np1; i += blockDim.x)
            ph_post[i] = ldg(ph + (size_t)(in.ph0 + post) * np1 + i);
}

// ---------------------------------------------------------------------------
// low pass: tile of 4096 contiguous amplitudes, 256 threads x 16 registers
// ---------------------------------------------------------------------------
constexpr int kLowBits = 12;
constexpr int kLowThreads = 256;

// LDS address swizzle: flips bits 0..3 by bits 4..7 and bit 4 by bit 8, so the
// three access patterns below hit distinct banks within each half wave.
__device__ __forceinline__ int swz(int i) { return i ^ ((i >> 4) & 15) ^ (((i >> 8) & 1) << 4); }

template <typename T>
__global__ __launch_bounds__(kLowThreads) void k_low(const DevInst *__restrict__ insts, int step,
                                                     int pre, int post, int n_plaq)
{
    using C = cplx_t<T>;
    __shared__ C buf[1 << kLowBits];
    __shared__ uint32_t ptab[kPtabWords];
    __shared__ C ph_pre[kMaxPlaq + 1], ph_post[kMaxPlaq + 1];

    const DevInst in = insts[blockIdx.y];
    if (in.step0 + step >= in.n_total) return;   // instance already finished (uniform per block)
    const gp<C> psi = (gp<C>)in.psi;
    const int t = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x << kLowBits;
    const RotParam<T> rp = ldg((gp<const RotParam<T>>)in.rot + (in.step0 + step));
    load_tables<T>(in, n_plaq, pre, post, ptab, ph_pre, ph_post);
    __syncthreads();

    C v[16];
    // stage 1: registers hold tile bits 8..11, coalesced loads
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = ldg(psi + (base + t + (r << 8)));
    if (pre >= 0) {
        uint32_t qs[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) qs[k] = link_set(8 + k, ptab);
        apply_phase_regs<C, 4>(v, syndrome(base + t, ptab), qs, ph_pre);
    }
    rot_regs<T, C, 4>(v, rp.u, rp.v);
#pragma unroll
    for (int r = 0; r < 16; ++r) buf[swz(t + (r << 8))] = v[r];
    __syncthreads();
    // stage 2: registers hold tile bits 4..7
    const int i2 = (t & 15) | ((t >> 4) << 8);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = buf[swz(i2 | (r << 4))];
    rot_regs<T, C, 4>(v, rp.u, rp.v);
#pragma unroll
    for (int r = 0; r < 16; ++r) buf[swz(i2 | (r << 4))] = v[r];
    __syncthreads();
    // stage 3: registers hold tile bits 0..3
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = buf[swz(r | (t << 4))];
    rot_regs<T, C, 4>(v, rp.u, rp.v);
    if (post >= 0) {
        uint32_t qs[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) qs[k] = link_set(k, ptab);
        apply_phase_regs<C, 4>(v, syndrome(base + ((uint64_t)t << 4), ptab), qs, ph_post);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) stg(psi + (base + ((uint64_t)t << 4) + r), v[r]);
}

// ---------------------------------------------------------------------------
// persistent tile pass.  A workgroup of 2^W waves owns tiles of 2^(10+W) amplitudes
// and walks over the tiles of its instance with a stride of gridDim.x, loading the
// next tile into registers while it works on the current one.
//   low tile:  tile bit i = index bit i, all 10+W bits rotated.
//   high tile: tile bits 0..CB-1 = index bits 0..CB-1 (rows of 2^CB amplitudes, not
//              rotated), tile bit i >= CB = index bit hb + i - CB (rotated).
// Layouts and the exchange between them are described at k_tile.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL,
                                                              0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double dpp_f(double x)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// value held by lane ^ (1 << B)
template <int B, typename T>
__device__ __forceinline__ T lane_partner(T x)
{
    if constexpr (B == 0) return dpp_f<0xB1>(x);                 // quad_perm [1,0,3,2]
    else if constexpr (B == 1) return dpp_f<0x4E>(x);            // quad_perm [2,3,0,1]
    else if constexpr (B == 2) return dpp_f<0x1B>(dpp_f<0x141>(x));  // half-row mirror, then ^3
    else if constexpr (B == 3) return dpp_f<0x128>(x);           // row_ror:8
    else return __shfl_xor(x, 1 << B, 64);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// a <- u a + i v a_partner for every register, partner across lane bit B.  tv / ntv hold
// t and -t in vector registers, so the cross-lane move can fold into the multiply-add.
// acc + src[partner lane] * mul, the lane permutation applied to src inside the multiply-
// add (DPP operand of v_fmac_f32).  The s_nop gives the two wait states a DPP read needs
// after a vector write of its source register.
template <int B>
__device__ __forceinline__ float fmac_partner(float acc, float src, float mul)
{
    if constexpr (B == 0)
        asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf"
            : "+v"(acc) : "v"(src), "v"(mul));
    else if constexpr (B == 1)
        asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf"
            : "+v"(acc) : "v"(src), "v"(mul));
    else if constexpr (B == 2)   // src already half-row mirrored: lane ^ 4 = mirror then ^ 3
        asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 quad_perm:[3,2,1,0] row_mask:0xf bank_mask:0xf"
            : "+v"(acc) : "v"(src), "v"(mul));
    else
        asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_ror:8 row_mask:0xf bank_mask:0xf"
            : "+v"(acc) : "v"(src), "v"(mul));
    return acc;
}

template <int B, bool TAN, typename T, typename C>
__device__ __forceinline__ void rot_lane(C *v, T tv, T ntv)
{
    if constexpr (TAN && sizeof(T) == 4 && B < 4) {
        // x' = x - t y[partner], y' = y + t x[partner]: one permutation rides in a
        // multiply-add, the other (of the value the first one overwrites) is a move
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if constexpr (B == 2) {
                const T mx = dpp_f<0x141>(v[r].x), my = dpp_f<0x141>(v[r].y);
                v[r].x = fmac_partner<2>(v[r].x, my, ntv);
                v[r].y = fmac_partner<2>(v[r].y, mx, tv);
            } else {
                const T pi = lane_partner<B>(v[r].y);
                v[r].y = fmac_partner<B>(v[r].y, v[r].x, tv);
                v[r].x = fma_t(ntv, pi, v[r].x);
            }
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const T pr = lane_partner<B>(v[r].x), pi = lane_partner<B>(v[r].y);
        if constexpr (TAN) {
            v[r].x = fma_t(ntv, pi, v[r].x);
            v[r].y = fma_t(tv, pr, v[r].y);
        } else {
            v[r].x = fma_t(tv, v[r].x, -pi);
            v[r].y = fma_t(tv, v[r].y, pr);
        }
    }
}

// pair update specialised for u = 1 (TAN) or v = 1
template <bool TAN, typename T, typename C>
__device__ __forceinline__ void rot_pair_s(C &a0, C &a1, T t)
{
    C b0, b1;
    if constexpr (TAN) {
        b0.x = a0.x - t * a1.y;
        b0.y = a0.y + t * a1.x;
        b1.x = a1.x - t * a0.y;
        b1.y = a1.y + t * a0.x;
    } else {
        b0.x = t * a0.x - a1.y;
        b0.y = t * a0.y + a1.x;
        b1.x = t * a1.x - a0.y;
        b1.y = t * a1.y + a0.x;
    }
    a0 = b0;
    a1 = b1;
}

template <bool TAN, int MASK, typename T, typename C>
__device__ __forceinline__ void rot_regs_s(C *v, T t)
{
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (MASK & (1 << k))
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (!(r & (1 << k))) rot_pair_s<TAN, T, C>(v[r], v[r | (1 << k)], t);
}

template <bool TAN, int LMASK, typename T, typename C>
__device__ __forceinline__ void rot_lanes(C *v, T t)
{
    // keep t and -t in VGPRs (an empty asm hides their uniformity from the compiler)
    T tv = t, ntv = -t;
    if constexpr (sizeof(T) == 4) {
        asm volatile("" : "+v"(tv));
        asm volatile("" : "+v"(ntv));
    }
    if constexpr (LMASK & 1) rot_lane<0, TAN, T, C>(v, tv, ntv);
    if constexpr (LMASK & 2) rot_lane<1, TAN, T, C>(v, tv, ntv);
    if constexpr (LMASK & 4) rot_lane<2, TAN, T, C>(v, tv, ntv);
    if constexpr (LMASK & 8) rot_lane<3, TAN, T, C>(v, tv, ntv);
    if constexpr (LMASK & 16) rot_lane<4, TAN, T, C>(v, tv, ntv);
    if constexpr (LMASK & 32) rot_lane<5, TAN, T, C>(v, tv, ntv);
}

// TAN / TN: rotation form of step and step + 1.  MERGE: rotation of `step`, the phase
// `post`, the rotation of step + 1; an instance whose last step is `step` stops after the
// phase and runs in the launch with TN == TAN.  Otherwise: the phase `pre` (if >= 0),
// the rotation of `step`, the phase `post` (if >= 0).  NT: non-temporal stores.
template <typename T, int W, int ROWB, bool TAN, bool TN, bool MERGE, bool NT = false>
__global__ __launch_bounds__(64 << W) void k_tile(const DevInst *__restrict__ insts, int n, int hb,
                                                  int step, int pre, int post, int n_plaq)
{
    using C = cplx_t<T>;
    using G = PassGeom<T, W, ROWB>;
    using MG = MergeGeom<T, W, ROWB>;
    constexpr bool LOW = G::LOW;
    constexpr int TB = G::TB, CB = G::CB;
    constexpr MergeLayout M = MG::M;
    static_assert(MG::swz(0) == 0, "layout");
    __shared__ C buf[1 << TB];
    __shared__ uint32_t ptab[kPtabWords];
    __shared__ C ph_pre[MERGE ? 1 : kMaxPlaq + 1], ph_post[kMaxPlaq + 1];
    static_assert(MERGE || TN == TAN, "single-step passes have one form");

    const DevInst in = insts[blockIdx.y];
    if (in.step0 + step >= in.n_total) return;   // instance already finished (uniform per block)
    const gp<const RotParam<T>> rot = (gp<const RotParam<T>>)in.rot;
    const RotParam<T> rp = ldg(rot + (in.step0 + step));
    if ((rp.u == T(1)) != TAN) return;           // the other form pairs have their own launches
    const T tt = TAN ? rp.v : rp.u;
    T tn = tt;
    // merged and the instance has step + 1; else the pass stops after the phase
    const bool more = MERGE && in.step0 + step + 1 < in.n_total;
    if (more) {
        const RotParam<T> rq = ldg(rot + (in.step0 + step + 1));
        if ((rq.u == T(1)) != TN) return;
        tn = TN ? rq.v : rq.u;
    } else if (TN != TAN) {
        return;
    }
    const gp<C> psi = (gp<C>)in.psi;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t n_tiles = 1ull << (n - TB);
    const int lowb = LOW ? 0 : hb - CB;
    // Rows shorter than a 128-byte cache line (complex128 rows of 4 amplitudes) leave the
    // other half of each line to the tile next to it (tile index ^ 1).  Workgroups go to the
    // eight XCDs in turn, each with its own L2, so tiles t and t ^ 1 are placed on one XCD:
    // tile bit 0 comes from bit 3 of the walk index and bits 1..3 from bits 0..2, which makes
    // walk indices p and p ^ 8 (same XCD, same round) the two halves of every line.
    constexpr bool HALF_LINE_ROWS = !LOW && (sizeof(C) << CB) < 128;
    auto tile_of = [&](uint64_t p) -> uint64_t {
        if constexpr (HALF_LINE_ROWS) return (p & ~15ull) | ((p & 7) << 1) | ((p >> 3) & 1);
        else return p;
    };
    auto tile_base = [&](uint64_t walk) -> uint64_t {
        const uint64_t tile = tile_of(walk);
        if constexpr (LOW) return tile << TB;
        else return ((tile & ((1ull << lowb) - 1)) << CB) | ((tile >> lowb) << (hb + TB - CB));
    };
    auto spread = [&](int o) -> uint64_t {
        if constexpr (LOW) return (uint64_t)o;
        else return (uint64_t)(o & ((1 << CB) - 1)) | ((uint64_t)(o >> CB) << hb);
    };
    auto gbit = [&](int i) -> int { return (LOW || i < CB) ? i : hb + (i - CB); };
    const int oA = l | (w << 6), oB = MG::thrB(l, w);
    const int sA = MG::swz(oA), sB = MG::swz(oB);   // LDS slots of register 0
    const uint32_t thrA = (uint32_t)spread(oA), thrBg = (uint32_t)spread(oB);
    uint64_t tile = blockIdx.x;
    if (tile >= n_tiles) return;
    C v[16], nv[16];
    {
        const gp<const C> tp = psi + tile_base(tile);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = ldg(tp + spread(r << (6 + W)) + thrA);
    }
    const bool phased = MERGE || pre >= 0 || post >= 0;
    uint32_t pra[16], prb[16];
    if (phased) {
        load_tables<T>(in, n_plaq, MERGE ? -1 : pre, post, ptab, ph_pre, ph_post);
        __syncthreads();
        uint32_t qa[4], qb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            qa[k] = link_set(gbit(6 + W + k), ptab);
            qb[k] = link_set(gbit(M.reg[k]), ptab);
        }
        reg_sets(qa, pra);
        reg_sets(qb, prb);
    }
    // One tile.  The next tile (or, without one, 16 cached loads of this tile's first row,
    // so that every tile sees the same memory operations in flight) is loaded into `y` in
    // four groups of registers spread over the work: loads issued in one burst stall the
    // issuing waves once the memory queues are full, and the vector units idle meanwhile.
    auto work = [&](uint64_t t_id, C *x, C *y, uint64_t nxt) __attribute__((always_inline)) {
        const uint64_t base = tile_base(t_id);
        const bool real = nxt < n_tiles;
        const gp<const C> tq = psi + tile_base(real ? nxt : t_id);
        const uint32_t lo = real ? thrA : (uint32_t)l;
        auto fetch = [&](int g) __attribute__((always_inline)) {
#pragma unroll
            for (int r = 4 * g; r < 4 * g + 4; ++r)
                y[r] = ldg(tq + (real ? spread(r << (6 + W)) : 0) + lo);
        };
        fetch(0);
        if (!MERGE && pre >= 0) apply_phase_pr<C>(x, syndrome(base + thrA, ptab), pra, ph_pre);
        // before the phase: A lanes 0..3 (register by register) and A registers
        rot_lanes<TAN, M.al, T, C>(x, tt);
        rot_regs_s<TAN, 15, T, C>(x, tt);
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[sA + (r << (6 + W))] = x[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = buf[sB + MG::regB(r)];
        fetch(1);
        // before the phase: B registers and lanes holding A's wave bits and bits 4, 5
        rot_regs_s<TAN, M.br1, T, C>(x, tt);
        rot_lanes<TAN, M.bl, T, C>(x, tt);
        if (MERGE || post >= 0) apply_phase_pr<C>(x, syndrome(base + thrBg, ptab), prb, ph_post);
        fetch(2);
        if (more) {
            rot_regs_s<TN, 15, T, C>(x, tn);
            rot_lanes<TN, M.bl, T, C>(x, tn);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[sB + MG::regB(r)] = x[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = buf[sA + (r << (6 + W))];
        fetch(3);
        if (more) {
            rot_regs_s<TN, M.ar2, T, C>(x, tn);
            rot_lanes<TN, M.al, T, C>(x, tn);
        }
        const gp<C> tp = psi + base;
        if constexpr (NT) {
#pragma unroll
            for (int r = 0; r < 16; ++r) stg_nt(tp + spread(r << (6 + W)) + thrA, x[r]);
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) stg(tp + spread(r << (6 + W)) + thrA, x[r]);
        }
    };
    // two register buffers alternate.  The first tile is peeled so that every tile in the
    // loop follows the same sequence of memory operations on every path.
    uint64_t next = tile + gridDim.x;
    work(tile, v, nv, next);
    while (next < n_tiles) {
        tile = next;
        next = tile + gridDim.x;
        work(tile, nv, v, next);
        if (next >= n_tiles) break;
        tile = next;
        next = tile + gridDim.x;
        work(tile, v, nv, next);
    }
}

// ---------------------------------------------------------------------------
// Tile with one more rotated bit kept in registers.  The tile is that of k_tile's
// geometry <T, W, ROWB> taken twice: once with index bit R clear and once with it set,
// R the bit above the tile's rotated bits (TB for a low tile, hb+TB-CB for a high tile).
// A thread holds both halves in 32 registers and rotates bit R between them; the other
// bits are rotated as in k_tile, one half at a time through LDS.  With complex128 this
// gives a high tile of 11 bits over full 128-byte rows (k_tile needs 64-byte rows for 11
// bits) or a low tile of 14 bits, so a 24-link step is two passes either way.  The 32
// registers leave no room for a prefetch buffer: the next tile is loaded once the
// current one is stored.
// ---------------------------------------------------------------------------
constexpr int kRbStaggerSleeps = 25;   // s_sleep 8 (512 clocks) each

template <typename T, int W, int ROWB, bool TAN, bool TN, bool MERGE>
__global__ __launch_bounds__(64 << W) void k_tile_rb(const DevInst *__restrict__ insts, int n,
                                                     int hb, int step, int pre, int post,
                                                     int n_plaq)
{
    using C = cplx_t<T>;
    using G = PassGeom<T, W, ROWB>;
    using MG = MergeGeom<T, W, ROWB>;
    constexpr bool LOW = G::LOW;
    constexpr int TB = G::TB, CB = G::CB;
    constexpr MergeLayout M = MG::M;
    __shared__ C buf[1 << TB];
    __shared__ uint32_t ptab[kPtabWords];
    __shared__ C ph_pre[MERGE ? 1 : kMaxPlaq + 1], ph_post[kMaxPlaq + 1];
    static_assert(MERGE || TN == TAN, "single-step passes have one form");

    const DevInst in = insts[blockIdx.y];
    if (in.step0 + step >= in.n_total) return;
    const gp<const RotParam<T>> rot = (gp<const RotParam<T>>)in.rot;
    const RotParam<T> rp = ldg(rot + (in.step0 + step));
    if ((rp.u == T(1)) != TAN) return;
    const T tt = TAN ? rp.v : rp.u;
    T tn = tt;
    const bool more = MERGE && in.step0 + step + 1 < in.n_total;
    if (more) {
        const RotParam<T> rq = ldg(rot + (in.step0 + step + 1));
        if ((rq.u == T(1)) != TN) return;
        tn = TN ? rq.v : rq.u;
    } else if (TN != TAN) {
        return;
    }
    const gp<C> psi = (gp<C>)in.psi;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rbit = LOW ? TB : hb + TB - CB;             // the register bit R
    const uint64_t n_tiles = 1ull << (n - TB - 1);
    const int lowb = LOW ? 0 : hb - CB;
    auto tile_base = [&](uint64_t tile) -> uint64_t {
        if constexpr (LOW) return tile << (TB + 1);
        else return ((tile & ((1ull << lowb) - 1)) << CB) | ((tile >> lowb) << (rbit + 1));
    };
    auto spread = [&](int o) -> uint64_t {
        if constexpr (LOW) return (uint64_t)o;
        else return (uint64_t)(o & ((1 << CB) - 1)) | ((uint64_t)(o >> CB) << hb);
    };
    auto gbit = [&](int i) -> int { return (LOW || i < CB) ? i : hb + (i - CB); };
    const int oA = l | (w << 6), oB = MG::thrB(l, w);
    const int sA = MG::swz(oA), sB = MG::swz(oB);
    const uint32_t thrA = (uint32_t)spread(oA), thrBg = (uint32_t)spread(oB);
    const uint64_t rofs = 1ull << rbit;
    const bool phased = MERGE || pre >= 0 || post >= 0;
    uint32_t pra[16], prb[16], qR = 0;
    if (phased) {
        load_tables<T>(in, n_plaq, MERGE ? -1 : pre, post, ptab, ph_pre, ph_post);
        __syncthreads();
        uint32_t qa[4], qb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            qa[k] = link_set(gbit(6 + W + k), ptab);
            qb[k] = link_set(gbit(M.reg[k]), ptab);
        }
        reg_sets(qa, pra);
        reg_sets(qb, prb);
        qR = link_set(rbit, ptab);
    }
    C x[32];
    // A tile's halves go through LDS one after the other: both to layout B (the rotations of
    // `step` before the exchange and after it), then bit R and the phase on both halves
    // in registers, then each half back to layout A and out.  A half's registers take the
    // next tile's loads as soon as that half is stored, so its loads run under the other
    // half's arithmetic and under the first half of the next tile.
    // All workgroups start together and would keep loading at the same time and computing
    // at the same time; half of the workgroups of each XCD (walk bit 3) start about
    // kRbStaggerSleeps x 512 clocks later, so that one half loads while the other computes.
    if (n_tiles > gridDim.x && ((blockIdx.x >> 3) & 1))
        for (int i = 0; i < kRbStaggerSleeps; ++i) __builtin_amdgcn_s_sleep(8);
    uint64_t tile = blockIdx.x;
    if (tile >= n_tiles) return;
    auto load_half = [&](uint64_t t_id, int h) __attribute__((always_inline)) {
        const gp<const C> tq = (gp<const C>)psi + tile_base(t_id) + (h ? rofs : 0);
#pragma unroll
        for (int r = 0; r < 16; ++r) x[16 * h + r] = ldg(tq + spread(r << (6 + W)) + thrA);
    };
    load_half(tile, 0);
    load_half(tile, 1);
    for (;;) {
        const uint64_t base = tile_base(tile), next = tile + gridDim.x;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            C *y = x + 16 * h;
            if (!MERGE && pre >= 0)
                apply_phase_pr<C>(y, syndrome(base + thrA, ptab) ^ (h ? qR : 0u), pra, ph_pre);
            rot_lanes<TAN, M.al, T, C>(y, tt);
            rot_regs_s<TAN, 15, T, C>(y, tt);
            // the first half writes exactly the slots this thread read last; the second
            // half's slots may still be read by other threads as their B slots
            if (h) __syncthreads();
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[sA + (r << (6 + W))] = y[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 16; ++r) y[r] = buf[sB + MG::regB(r)];
            rot_regs_s<TAN, M.br1, T, C>(y, tt);
            rot_lanes<TAN, M.bl, T, C>(y, tt);
        }
        // bit R, the phase, and bit R of step + 1: both halves in layout B
#pragma unroll
        for (int r = 0; r < 16; ++r) rot_pair_s<TAN, T, C>(x[r], x[16 + r], tt);
        if (MERGE || post >= 0) {
            const uint32_t P0 = syndrome(base + thrBg, ptab);
            apply_phase_pr<C>(x, P0, prb, ph_post);
            apply_phase_pr<C>(x + 16, P0 ^ qR, prb, ph_post);
        }
        if (more) {
#pragma unroll
            for (int r = 0; r < 16; ++r) rot_pair_s<TN, T, C>(x[r], x[16 + r], tn);
        }
        // the store addresses are formed again here: kept from the loads they would hold
        // 64 more registers through the tile
        uint64_t sbase = base;
        asm volatile("" : "+s"(sbase));
        const gp<C> sp = psi + sbase;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            C *y = x + 16 * h;
            if (more) {
                rot_regs_s<TN, 15, T, C>(y, tn);
                rot_lanes<TN, M.bl, T, C>(y, tn);
            }
            // the first half writes the B slots this thread read last; the second half's
            // may still be read by other threads as their A slots
            if (h) __syncthreads();
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[sB + MG::regB(r)] = y[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 16; ++r) y[r] = buf[sA + (r << (6 + W))];
            if (more) {
                rot_regs_s<TN, M.ar2, T, C>(y, tn);
                rot_lanes<TN, M.al, T, C>(y, tn);
            }
            const gp<C> hp = sp + (h ? rofs : 0);
#pragma unroll
            for (int r = 0; r < 16; ++r) stg(hp + spread(r << (6 + W)) + thrA, y[r]);
            if (next < n_tiles) load_half(next, h);
        }
        if (next >= n_tiles) break;
        tile = next;
    }
}

// ---------------------------------------------------------------------------
// high pass: link qubits [q0, q0+H) from registers, lanes on consecutive amplitudes
// ---------------------------------------------------------------------------
constexpr int kHighThreads = 256;

template <typename T, int H>
__global__ __launch_bounds__(kHighThreads) void k_high(const DevInst *__restrict__ insts, int q0,
                                                       int step, int post, int n_plaq)
{
    using C = cplx_t<T>;
    __shared__ uint32_t ptab[kPtabWords];
    __shared__ C ph_post[kMaxPlaq + 1];
    const DevInst in = insts[blockIdx.y];
    if (in.step0 + step >= in.n_total) return;   // instance already finished (uniform per block)
    const gp<C> psi = (gp<C>)in.psi;
    const RotParam<T> rp = ldg((gp<const RotParam<T>>)in.rot + (in.step0 + step));
    if (post >= 0) {
        load_tables<T>(in, n_plaq, -1, post, ptab, nullptr, ph_post);
        __syncthreads();
    }
    const uint64_t g = (uint64_t)blockIdx.x * kHighThreads + threadIdx.x;
    const uint64_t lowmask = (1ull << q0) - 1;
    const uint64_t base = (g & lowmask) | ((g >> q0) << (q0 + H));
    C v[1 << H];
#pragma unroll
    for (int r = 0; r < (1 << H); ++r) v[r] = ldg(psi + (base + ((uint64_t)r << q0)));
    rot_regs<T, C, H>(v, rp.u, rp.v);
    if (post >= 0) {
        uint32_t qs[H];
#pragma unroll
        for (int k = 0; k < H; ++k) qs[k] = link_set(q0 + k, ptab);
        apply_phase_regs<C, H>(v, syndrome(base, ptab), qs, ph_post);
    }
#pragma unroll
    for (int r = 0; r < (1 << H); ++r) stg(psi + (base + ((uint64_t)r << q0)), v[r]);
}

// ---------------------------------------------------------------------------
// standalone plaquette phase: 16 consecutive amplitudes per thread
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_phase(const DevInst *__restrict__ insts, int n,
                                               int idx, int n_plaq)
{
    using C = cplx_t<T>;
    __shared__ uint32_t ptab[kPtabWords];
    __shared__ C ph[kMaxPlaq + 1];
    const DevInst in = insts[blockIdx.y];
    load_tables<T>(in, n_plaq, -1, idx, ptab, nullptr, ph);
    __syncthreads();
    const gp<C> psi = (gp<C>)in.psi;
    const uint64_t dim = 1ull << n;
    const int nb = n < 4 ? n : 4;
    uint32_t qs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) qs[k] = (k < nb) ? link_set(k, ptab) : 0u;
    for (uint64_t base = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) << 4; base < dim;
         base += ((uint64_t)gridDim.x * blockDim.x) << 4) {
        const uint32_t P0 = syndrome(base, ptab);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (r < (1 << nb)) {
                uint32_t P = P0;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (r & (1 << k)) P ^= qs[k];
                stg(psi + (base + r), cmul_ph(ldg(psi + (base + r)), ph[__popc(P)]));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// small states (n <= 12): the whole evolution of one instance in one workgroup,
// state resident in LDS for every step of the call
// ---------------------------------------------------------------------------
constexpr int kSmallThreads = 256;

template <typename T>
__global__ __launch_bounds__(kSmallThreads) void k_small(const DevInst *__restrict__ insts, int n,
                                                         int n_steps, int pre, int n_plaq)
{
    using C = cplx_t<T>;
    __shared__ C a[1 << 12];
    __shared__ uint32_t ptab[kPtabWords];
    __shared__ uint8_t syn[1 << 12];
    __shared__ C ph[kMaxPlaq + 1];
    const DevInst in = insts[blockIdx.x];
    const gp<C> psi = (gp<C>)in.psi;
    const int dim = 1 << n, t = threadIdx.x;
    const int np1 = n_plaq + 1;
    const gp<const C> phase = (gp<const C>)in.phase;
    const gp<const RotParam<T>> rot = (gp<const RotParam<T>>)in.rot;
    for (int i = t; i < kPtabWords; i += kSmallThreads) ptab[i] = ((gp<const uint32_t>)in.ptab)[i];
    __syncthreads();
    for (int b = t; b < dim; b += kSmallThreads) {
        a[b] = ldg(psi + b);
        syn[b] = (uint8_t)__popc(syndrome((uint64_t)b, ptab));
    }
    int k = in.ph0;
    const int steps = min(n_steps, in.n_total - in.step0);
    if (pre) {
        for (int i = t; i < np1; i += kSmallThreads) ph[i] = ldg(phase + ((size_t)k * np1 + i));
        __syncthreads();
        for (int b = t; b < dim; b += kSmallThreads) a[b] = cmul_ph(a[b], ph[syn[b]]);
        ++k;
    }
    __syncthreads();
    for (int j = 0; j < steps; ++j, ++k) {
        const RotParam<T> rp = ldg(rot + (in.step0 + j));
        for (int q = 0; q < n; ++q) {
            const int lo = (1 << q) - 1;
            for (int p = t; p < (dim >> 1); p += kSmallThreads) {
                const int i0 = ((p & ~lo) << 1) | (p & lo);
                rot_pair<T, C>(a[i0], a[i0 | (1 << q)], rp.u, rp.v);
            }
            __syncthreads();
        }
        for (int i = t; i < np1; i += kSmallThreads) ph[i] = ldg(phase + ((size_t)k * np1 + i));
        __syncthreads();
        for (int b = t; b < dim; b += kSmallThreads) a[b] = cmul_ph(a[b], ph[syn[b]]);
        __syncthreads();
    }
    for (int b = t; b < dim; b += kSmallThreads) stg(psi + b, a[b]);
}

// ---------------------------------------------------------------------------
// wave-resident states (6 + RB <= 8 links): one wavefront per instance holds the whole
// state, lanes on index bits 0..5 and 2^RB registers on bits 6..5+RB, for every step
// of the call; rotations across lanes and registers, no LDS traffic but the phase table
// ---------------------------------------------------------------------------
template <int B, bool TAN, int R, typename T, typename C>
__device__ __forceinline__ void rot_lane_r(C *v, T t)
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const T pr = lane_partner<B>(v[r].x), pi = lane_partner<B>(v[r].y);
        if constexpr (TAN) {
            v[r].x = v[r].x - t * pi;
            v[r].y = v[r].y + t * pr;
        } else {
            v[r].x = t * v[r].x - pi;
            v[r].y = t * v[r].y + pr;
        }
    }
}

template <bool TAN, int RB, typename T, typename C>
__device__ __forceinline__ void wave_layer(C *v, T t)
{
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int r = 0; r < (1 << RB); ++r)
            if (!(r & (1 << k))) rot_pair_s<TAN, T, C>(v[r], v[r | (1 << k)], t);
    rot_lane_r<0, TAN, 1 << RB, T, C>(v, t);
    rot_lane_r<1, TAN, 1 << RB, T, C>(v, t);
    rot_lane_r<2, TAN, 1 << RB, T, C>(v, t);
    rot_lane_r<3, TAN, 1 << RB, T, C>(v, t);
    rot_lane_r<4, TAN, 1 << RB, T, C>(v, t);
    rot_lane_r<5, TAN, 1 << RB, T, C>(v, t);
}

template <typename T, int RB>
__global__ __launch_bounds__(64) void k_wave(const DevInst *__restrict__ insts, int n_steps,
                                             int pre, int n_plaq)
{
    using C = cplx_t<T>;
    constexpr int R = 1 << RB;
    __shared__ uint32_t ptab[kPtabWords];
    __shared__ C ph[kMaxPlaq + 1];
    const DevInst in = insts[blockIdx.x];
    const gp<C> psi = (gp<C>)in.psi;
    const int l = threadIdx.x, np1 = n_plaq + 1;
    const gp<const C> phase = (gp<const C>)in.phase;
    const gp<const RotParam<T>> rot = (gp<const RotParam<T>>)in.rot;
    for (int i = l; i < kPtabWords; i += 64) ptab[i] = ((gp<const uint32_t>)in.ptab)[i];
    __syncthreads();
    C v[R];
    int m[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        v[r] = ldg(psi + (l | (r << 6)));
        m[r] = __popc(syndrome((uint64_t)(l | (r << 6)), ptab));
    }
    auto phase_step = [&](int k) {
        if (l < np1) ph[l] = ldg(phase + ((size_t)k * np1 + l));
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = cmul_ph(v[r], ph[m[r]]);
        __syncthreads();
    };
    int k = in.ph0;
    const int steps = min(n_steps, in.n_total - in.step0);
    if (pre) phase_step(k++);
    for (int j = 0; j < steps; ++j, ++k) {
        const RotParam<T> rp = ldg(rot + (in.step0 + j));
        if (rp.u == T(1)) wave_layer<true, RB, T, C>(v, rp.v);
        else wave_layer<false, RB, T, C>(v, rp.u);
        phase_step(k);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) stg(psi + (l | (r << 6)), v[r]);
}

// ---------------------------------------------------------------------------
// state preparation
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_init(cplx_t<T> *psi, int n, int init, uint64_t basis, T amp,
                       const uint32_t *__restrict__ ptab)
{
    const uint64_t dim = 1ull << n;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < dim;
         b += (uint64_t)gridDim.x * blockDim.x) {
        cplx_t<T> v;
        v.y = 0;
        if (init == LGT_INIT_PLUS) v.x = amp;
        else if (init == LGT_INIT_BASIS) v.x = (b == basis) ? T(1) : T(0);
        else v.x = syndrome(b, ptab) == 0u ? amp : T(0);
        psi[b] = v;
    }
}

// ---------------------------------------------------------------------------
// circuit-form gates, one full-state pass each (eq. (ara) and the R_x layer)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_gate_h(cplx_t<T> *psi, int n, int q)
{
    // Hadamard on link q: (a0, a1) <- ((a0 + a1) / sqrt 2, (a0 - a1) / sqrt 2)
    const T r = T(0.70710678118654752440);
    const uint64_t half = 1ull << (n - 1), lo = (1ull << q) - 1;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < half;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i0 = ((p & ~lo) << 1) | (p & lo), i1 = i0 | (lo + 1);
        const cplx_t<T> a0 = psi[i0], a1 = psi[i1];
        cplx_t<T> b0, b1;
        b0.x = (a0.x + a1.x) * r;
        b0.y = (a0.y + a1.y) * r;
        b1.x = (a0.x - a1.x) * r;
        b1.y = (a0.y - a1.y) * r;
        psi[i0] = b0;
        psi[i1] = b1;
    }
}

// (X^x Z^z psi)_b = (-1)^popcount((b ^ x) & z) psi_{b ^ x}; pairs (b, b ^ x) are handled by
// the thread whose b has a zero at the lowest bit of x (x != 0), single amplitudes otherwise
template <typename T>
__global__ void k_pauli(cplx_t<T> *psi, int n, uint64_t x, uint64_t z)
{
    using C = cplx_t<T>;
    auto sgn = [&](uint64_t b) -> T { return (__popcll(b & z) & 1) ? T(-1) : T(1); };
    if (x == 0) {
        for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < (1ull << n);
             b += (uint64_t)gridDim.x * blockDim.x) {
            C a = psi[b];
            const T s = sgn(b);
            a.x *= s;
            a.y *= s;
            psi[b] = a;
        }
        return;
    }
    const uint64_t lo = (x & (~x + 1)) - 1;   // bits below the lowest set bit of x
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < (1ull << (n - 1));
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t b = ((p & ~lo) << 1) | (p & lo), c = b ^ x;
        C a0 = psi[b], a1 = psi[c];
        const T s0 = sgn(c), s1 = sgn(b);
        C r0, r1;
        r0.x = s0 * a1.x;
        r0.y = s0 * a1.y;
        r1.x = s1 * a0.x;
        r1.y = s1 * a0.y;
        psi[b] = r0;
        psi[c] = r1;
    }
}

template <typename T>
__global__ void k_gate_rx(cplx_t<T> *psi, int n, int q, T c, T s)
{
    // R_x(phi) = exp(-i sigma^x phi/2): (a0, a1) <- (c a0 - i s a1, -i s a0 + c a1)
    const uint64_t half = 1ull << (n - 1), lo = (1ull << q) - 1;
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < half;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i0 = ((p & ~lo) << 1) | (p & lo), i1 = i0 | (lo + 1);
        cplx_t<T> a0 = psi[i0], a1 = psi[i1], b0, b1;
        // the products with c (within a few ulps of 1 for small angles) stay inside the FMA
        b0.x = fma_r(c, a0.x, s * a1.y);
        b0.y = fma_r(c, a0.y, -(s * a1.x));
        b1.x = fma_r(c, a1.x, s * a0.y);
        b1.y = fma_r(c, a1.y, -(s * a0.x));
        psi[i0] = b0;
        psi[i1] = b1;
    }
}

template <typename T>
__global__ void k_gate_rz(cplx_t<T> *psi, int n, int q, cplx_t<T> e0, cplx_t<T> e1)
{
    const uint64_t dim = 1ull << n;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < dim;
         b += (uint64_t)gridDim.x * blockDim.x)
        psi[b] = cmul_ph(psi[b], ((b >> q) & 1) ? e1 : e0);
}

// controlled-Z: sign flip where qubits a and b are both |1>
template <typename T>
__global__ void k_gate_cz(cplx_t<T> *psi, int n, uint64_t both)
{
    const uint64_t dim = 1ull << n;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < dim;
         b += (uint64_t)gridDim.x * blockDim.x)
        if ((b & both) == both) {
            cplx_t<T> a = psi[b];
            a.x = -a.x;
            a.y = -a.y;
            psi[b] = a;
        }
}

// measurement with outcome |0> on every qubit of zero_mask (those amplitudes dropped),
// the rest multiplied by `scale`
template <typename T>
__global__ void k_project_scale(cplx_t<T> *psi, int n, uint64_t zero_mask, T scale)
{
    const uint64_t dim = 1ull << n;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < dim;
         b += (uint64_t)gridDim.x * blockDim.x) {
        cplx_t<T> a = psi[b];
        if (b & zero_mask) {
            a.x = 0;
            a.y = 0;
        } else {
            a.x *= scale;
            a.y *= scale;
        }
        psi[b] = a;
    }
}

template <typename T>
__global__ void k_gate_cnot(cplx_t<T> *psi, int n, int c, int t)
{
    // swap the pair (b, b ^ 2^t) for every b with control bit set and target bit clear
    const int lo_b = c < t ? c : t, hi_b = c < t ? t : c;
    const uint64_t quarter = 1ull << (n - 2);
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < quarter;
         p += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t i = p;
        i = ((i >> lo_b) << (lo_b + 1)) | (i & ((1ull << lo_b) - 1));
        i = ((i >> hi_b) << (hi_b + 1)) | (i & ((1ull << hi_b) - 1));
        i |= 1ull << c;
        const uint64_t j = i | (1ull << t);
        cplx_t<T> x = psi[i];
        psi[i] = psi[j];
        psi[j] = x;
    }
}

// ---------------------------------------------------------------------------
// FP64 reductions (Sec. 2.4: sums over all basis states)
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 256;
constexpr int kRedMasks = 32;     // masks per diagonal launch
constexpr int kFlipMasks = 8;     // masks per off-diagonal launch

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// block-level sum of acc[M] into out[M] (deterministic order)
template <int M>
__device__ __forceinline__ void block_sum_store(double *acc, double *out)
{
    __shared__ double red[kRedThreads / 64][M];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double s = wave_sum(acc[m]);
        if (lane == 0) red[w][m] = s;
    }
    __syncthreads();
    for (int m = threadIdx.x; m < M; m += kRedThreads) {
        double s = 0;
        for (int k = 0; k < kRedThreads / 64; ++k) s += red[k][m];
        out[m] = s;
    }
}

// acc[m] += |psi_b|^2 * (-1)^{popcount(b & mask_m)}.  The index splits as
// b = tid | blk << 8 | k << (8 + GB) | o << (8 + GB + KB) (2^GB = gridDim.x).  For each o a
// thread holds the 2^KB probabilities p_k and takes their Walsh-Hadamard transform
// W_f = sum_k (-1)^{popcount(k & f)} p_k, so mask m needs only W at f = its k bits (read
// back from the thread's own LDS column), times the sign of its o bits, which is the same
// across the block; the sign of its tid and blk bits is applied once at the end.
template <typename T, int KB>
__global__ __launch_bounds__(kRedThreads) void k_red_diag(const cplx_t<T> *__restrict__ psi, int n,
                                                          const uint64_t *__restrict__ masks,
                                                          int n_masks, double *partials)
{
    static_assert(kRedThreads == 256, "eight index bits per thread");
    constexpr int K = 1 << KB;
    __shared__ double wl[K][kRedThreads];
    const uint32_t tid = threadIdx.x;
    const int kshift = 8 + (31 - __builtin_clz(gridDim.x)), oshift = kshift + KB;
    const uint64_t n_o = (1ull << n) >> oshift;
    const uint64_t base = tid | ((uint64_t)blockIdx.x << 8);
    uint64_t mh[kRedMasks];
#pragma unroll
    for (int m = 0; m < kRedMasks; ++m) mh[m] = m < n_masks ? masks[m] : 0;
    double acc[kRedMasks];
#pragma unroll
    for (int m = 0; m < kRedMasks; ++m) acc[m] = 0;
    for (uint64_t o = 0; o < n_o; ++o) {
        double w[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const cplx_t<T> a = psi[base | ((uint64_t)k << kshift) | (o << oshift)];
            w[k] = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
        }
#pragma unroll
        for (int h = 1; h < K; h <<= 1)
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (!(i & h)) {
                    const double x = w[i], y = w[i | h];
                    w[i] = x + y;
                    w[i | h] = x - y;
                }
#pragma unroll
        for (int f = 0; f < K; ++f) wl[f][tid] = w[f];
#pragma unroll
        for (int m = 0; m < kRedMasks; ++m) {
            const int f = (int)((mh[m] >> kshift) & (uint64_t)(K - 1));
            const double so = (__popcll(o & (mh[m] >> oshift)) & 1) ? -1.0 : 1.0;
            acc[m] = __builtin_fma(so, wl[f][tid], acc[m]);
        }
    }
#pragma unroll
    for (int m = 0; m < kRedMasks; ++m)
        if (__popcll(base & mh[m]) & 1) acc[m] = -acc[m];
    block_sum_store<kRedMasks>(acc, partials + (size_t)blockIdx.x * kRedMasks);
}

// acc[m] += Re conj(psi_b) psi_{b ^ mask_m}
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_red_flip(const cplx_t<T> *__restrict__ psi, int n,
                                                          const uint64_t *__restrict__ masks,
                                                          int n_masks, double *partials)
{
    __shared__ uint64_t mk[kFlipMasks];
    if (threadIdx.x < kFlipMasks) mk[threadIdx.x] = threadIdx.x < n_masks ? masks[threadIdx.x] : 0;
    __syncthreads();
    double acc[kFlipMasks];
#pragma unroll
    for (int m = 0; m < kFlipMasks; ++m) acc[m] = 0;
    const uint64_t dim = 1ull << n;
    for (uint64_t b = (uint64_t)blockIdx.x * kRedThreads + threadIdx.x; b < dim;
         b += (uint64_t)gridDim.x * kRedThreads) {
        const cplx_t<T> a = psi[b];
#pragma unroll
        for (int m = 0; m < kFlipMasks; ++m) {
            if (m < n_masks) {
                const cplx_t<T> c = psi[b ^ mk[m]];
                acc[m] += (double)a.x * (double)c.x + (double)a.y * (double)c.y;
            }
        }
    }
    block_sum_store<kFlipMasks>(acc, partials + (size_t)blockIdx.x * kFlipMasks);
}

// out[c] = sum over rows of partials[row][c], c < ncols: one block per column, each thread
// sums a fixed set of rows, then a fixed-order block sum (the same result every call)
__global__ __launch_bounds__(kRedThreads) void k_sum_cols(const double *__restrict__ partials,
                                                          int rows, int width, double *out)
{
    const int c = blockIdx.x;
    double acc = 0;
    for (int r = threadIdx.x; r < rows; r += kRedThreads) acc += partials[(size_t)r * width + c];
    block_sum_store<1>(&acc, out + c);
}

// Z density of states: acc[m] += |psi_b|^2 for the m = popcount(P(b)) bin
// BYPOP: the bin is popcount(b) itself (a density of states in the basis of a transformed
// copy of the state), otherwise the number of odd plaquettes of b
template <typename T, bool BYPOP>
__global__ __launch_bounds__(kRedThreads) void k_red_dos(const cplx_t<T> *__restrict__ psi, int n,
                                                         const uint32_t *__restrict__ ptab_g,
                                                         int n_plaq, double *partials)
{
    __shared__ uint32_t ptab[kPtabWords];
    for (int i = threadIdx.x; i < kPtabWords; i += kRedThreads) ptab[i] = ptab_g[i];
    __syncthreads();
    double acc[kMaxPlaq + 1];
#pragma unroll
    for (int m = 0; m <= kMaxPlaq; ++m) acc[m] = 0;
    const uint64_t dim = 1ull << n;
    for (uint64_t b = (uint64_t)blockIdx.x * kRedThreads + threadIdx.x; b < dim;
         b += (uint64_t)gridDim.x * kRedThreads) {
        const cplx_t<T> a = psi[b];
        const double p = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
        const int m = BYPOP ? __popcll(b) : __popc(syndrome(b, ptab));
#pragma unroll
        for (int k = 0; k <= kMaxPlaq; ++k) acc[k] += (m == k) ? p : 0.0;
    }
    block_sum_store<kMaxPlaq + 1>(acc, partials + (size_t)blockIdx.x * (kMaxPlaq + 1));
}

// ---------------------------------------------------------------------------
// sampling: FP64 block sums, prefix, inverse CDF per shot
// ---------------------------------------------------------------------------
constexpr int kSampleBlockBits = 10;   // amplitudes per block sum

template <typename T>
__global__ __launch_bounds__(256) void k_block_sums(const cplx_t<T> *__restrict__ psi, int n,
                                                    double *sums)
{
    // one block sum of 2^kSampleBlockBits amplitudes per 256-thread group, in a fixed order
    __shared__ double red[256];
    const int bb = n < kSampleBlockBits ? n : kSampleBlockBits;
    const uint64_t base = (uint64_t)blockIdx.x << bb;
    double s = 0;
    for (int i = threadIdx.x; i < (1 << bb); i += 256) {
        const cplx_t<T> a = psi[base + i];
        s += (double)a.x * (double)a.x + (double)a.y * (double)a.y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__device__ __forceinline__ double splitmix_uniform(uint64_t seed, uint64_t i)
{
    // SplitMix64 finaliser on the counter seed + (i+1) * golden gamma
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_sample(const cplx_t<T> *__restrict__ psi, int n,
                                                const double *__restrict__ prefix, int n_blocks,
                                                uint64_t n_shots, uint64_t seed, uint64_t *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_shots) return;
    const double total = prefix[n_blocks - 1];
    const double target = splitmix_uniform(seed, i) * total;
    // first block whose inclusive prefix exceeds the target
    int lo = 0, hi = n_blocks - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] > target) hi = mid; else lo = mid + 1;
    }
    const int bb = n < kSampleBlockBits ? n : kSampleBlockBits;
    const uint64_t base = (uint64_t)lo << bb;
    double acc = lo > 0 ? prefix[lo - 1] : 0.0;
    uint64_t pick = base, last_nz = base;
    bool found = false;
    for (int k = 0; k < (1 << bb); ++k) {
        const cplx_t<T> a = psi[base + k];
        const double p = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
        if (p > 0) last_nz = base + k;
        acc += p;
        if (acc > target) {
            pick = base + k;
            found = true;
            break;
        }
    }
    out[i] = found ? pick : last_nz;
}

// inclusive prefix of the block sums in place, ascending, by one thread: the same additions
// in the same order as the host prefix of launch_sample, so both give the same bits
__global__ void k_prefix_seq(double *sums, int nb)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double acc = 0;
    for (int i = 0; i < nb; ++i) {
        acc += sums[i];
        sums[i] = acc;
    }
}

// ---------------------------------------------------------------------------
// scratch of the allocation-free sampling entry point: block sums (kScratchSums doubles)
// then shots (kScratchShots words).  One copy per device, held until the process ends.
// Host code never uses the array's name as an address: scratch_address() looks up the
// device address once per device with hipGetSymbolAddress.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint64_t scratch[kScratchSums + kScratchShots];

hipError_t scratch_address(int device, void **out)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
const char *kernel_family_name(int kf)
{
    static const char *names[KF_COUNT] = {"init", "pass_low", "pass_high", "phase", "small",
                                          "gate_rx", "gate_rz", "gate_cnot", "reduce_diag",
                                          "reduce_flip", "reduce_dos", "sample", "tile_low",
                                          "tile_high", "gate_h", "gate_cz", "project"};
    return (kf >= 0 && kf < KF_COUNT) ? names[kf] : "?";
}

static unsigned grid_for(uint64_t work, unsigned per_block, unsigned cap = 65536u)
{
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

hipError_t launch_init(int dtype, void *psi, int n, int init, uint64_t basis, double amp,
                       const uint32_t *ptab_dev, hipStream_t st)
{
    const unsigned g = grid_for(1ull << n, 256, 16384);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_init<float>, dim3(g), dim3(256), 0, st, (float2 *)psi, n, init,
                           basis, (float)amp, ptab_dev);
    else
        hipLaunchKernelGGL(k_init<double>, dim3(g), dim3(256), 0, st, (double2 *)psi, n, init,
                           basis, amp, ptab_dev);
    return hipGetLastError();
}

hipError_t launch_low(int dtype, const DevInst *dev_inst, int n_inst, int n, int low_bits,
                      int step, int pre, int post, int n_plaq, hipStream_t st)
{
    if (low_bits != kLowBits || n < kLowBits) return hipErrorInvalidValue;
    dim3 grid((unsigned)(1ull << (n - kLowBits)), (unsigned)n_inst);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_low<float>, grid, dim3(kLowThreads), 0, st, dev_inst, step, pre,
                           post, n_plaq);
    else
        hipLaunchKernelGGL(k_low<double>, grid, dim3(kLowThreads), 0, st, dev_inst, step, pre,
                           post, n_plaq);
    return hipGetLastError();
}

thread_local LaunchTiming *g_launch_timing = nullptr;

template <typename K, typename... A>
static void launch_timed(K kernel, dim3 g, dim3 b, hipStream_t st, A... args)
{
    LaunchTiming *lt = g_launch_timing;
    if (!lt) {
        hipLaunchKernelGGL(kernel, g, b, 0, st, args...);
        return;
    }
    hipExtLaunchKernelGGL(kernel, g, b, 0, st, lt->used ? nullptr : lt->start, lt->stop, 0, args...);
    lt->used = true;
}

template <typename T, int W, int ROWB, bool NT>
static hipError_t launch_pass_nt(const DevInst *dev_inst, int n, int hb, int step, int pre,
                                 int post, int n_plaq, int forms, int merge, dim3 g, dim3 b,
                                 hipStream_t st)
{
    if (merge) {
        // forms: bits 0-1 the forms of `step`, bits 2-3 those of step + 1; every form pair
        // that some instance may have gets a launch, and each instance runs in exactly one
        if (pre >= 0 || post < 0) return hipErrorInvalidValue;   // merged: one phase between
        const int fa = forms & 3, fb = (forms >> 2) & 3;
        if (fa & 1) {
            launch_timed(k_tile<T, W, ROWB, true, true, true, NT>, g, b, st, dev_inst, n, hb, step, -1, post, n_plaq);
            if (fb & 2)
                launch_timed(k_tile<T, W, ROWB, true, false, true, NT>, g, b, st, dev_inst, n, hb, step, -1, post, n_plaq);
        }
        if (fa & 2) {
            launch_timed(k_tile<T, W, ROWB, false, false, true, NT>, g, b, st, dev_inst, n, hb, step, -1, post, n_plaq);
            if (fb & 1)
                launch_timed(k_tile<T, W, ROWB, false, true, true, NT>, g, b, st, dev_inst, n, hb, step, -1, post, n_plaq);
        }
        return hipGetLastError();
    }
    if (forms & 1)
        launch_timed(k_tile<T, W, ROWB, true, true, false, NT>, g, b, st, dev_inst, n, hb, step, pre, post, n_plaq);
    if (forms & 2)
        launch_timed(k_tile<T, W, ROWB, false, false, false, NT>, g, b, st, dev_inst, n, hb, step, pre, post, n_plaq);
    return hipGetLastError();
}

template <typename T, int W, int ROWB>
static hipError_t launch_pass_t(const DevInst *dev_inst, int n_inst, int n, int hb, int step,
                                int pre, int post, int n_plaq, int forms, int merge, hipStream_t st)
{
    constexpr int TB = 10 + W;
    const uint64_t n_tiles = 1ull << (n - TB);
    // resident workgroups per CU: one for the 512- and 1024-thread tiles, else as many as
    // the 160 KiB of LDS holds, at most four (with two, batches of 21-64 18-link states ran
    // 6-7% slower); a batch splits the resident slots of the 256 CUs between its instances,
    // and each instance's tiles are spread evenly over as few workgroups as take the same
    // number of rounds
    constexpr uint64_t tile_bytes = (uint64_t)sizeof(cplx_t<T>) << TB;
    const uint64_t per_cu = (W >= 3) ? 1 : std::min<uint64_t>(4, (160ull << 10) / tile_bytes);
    uint64_t slots = 256 * per_cu / (uint64_t)n_inst;
    if (slots < 1) slots = 1;
    const uint64_t rounds = (n_tiles + slots - 1) / slots;
    const uint64_t grid = (n_tiles + rounds - 1) / rounds;
    const dim3 g((unsigned)grid, (unsigned)n_inst), b(64 << W);
    if constexpr (PassGeom<T, W, ROWB>::LOW) {
        // Low tiles of states too large to stay in the 256 MB Infinity Cache between passes
        // store non-temporally: 10-13% faster from 512 MiB on (28 and 32 links), slower at
        // 128-256 MiB, where the next pass finds the state in that cache.  High tiles gain
        // nothing from it (slower at 32 links).
        const uint64_t bytes = ((uint64_t)n_inst * sizeof(T) * 2) << n;
        if (bytes >= (512ull << 20))
            return launch_pass_nt<T, W, ROWB, true>(dev_inst, n, hb, step, pre, post, n_plaq, forms, merge, g, b, st);
    }
    return launch_pass_nt<T, W, ROWB, false>(dev_inst, n, hb, step, pre, post, n_plaq, forms, merge, g, b, st);
}

// the register-bit tiles (k_tile_rb): one resident workgroup per CU, tiles of 2^(TB+1)
template <typename T, int W, int ROWB>
static hipError_t launch_pass_rb(const DevInst *dev_inst, int n_inst, int n, int hb, int step,
                                 int pre, int post, int n_plaq, int forms, int merge,
                                 hipStream_t st)
{
    constexpr int TB = 10 + W;
    const uint64_t n_tiles = 1ull << (n - TB - 1);
    uint64_t slots = 256 / (uint64_t)n_inst;
    if (slots < 1) slots = 1;
    const uint64_t rounds = (n_tiles + slots - 1) / slots;
    const uint64_t grid = (n_tiles + rounds - 1) / rounds;
    const dim3 g((unsigned)grid, (unsigned)n_inst), b(64 << W);
    if (merge) {
        if (pre >= 0 || post < 0) return hipErrorInvalidValue;
        const int fa = forms & 3, fb = (forms >> 2) & 3;
        if (fa & 1) {
            launch_timed(k_tile_rb<T, W, ROWB, true, true, true>, g, b, st, dev_inst, n, hb, step, -1, post, n_plaq);
            if (fb & 2)
                launch_timed(k_tile_rb<T, W, ROWB, true, false, true>, g, b, st, dev_inst, n, hb, step, -1, post, n_plaq);
        }
        if (fa & 2) {
            launch_timed(k_tile_rb<T, W, ROWB, false, false, true>, g, b, st, dev_inst, n, hb, step, -1, post, n_plaq);
            if (fb & 1)
                launch_timed(k_tile_rb<T, W, ROWB, false, true, true>, g, b, st, dev_inst, n, hb, step, -1, post, n_plaq);
        }
        return hipGetLastError();
    }
    if (forms & 1)
        launch_timed(k_tile_rb<T, W, ROWB, true, true, false>, g, b, st, dev_inst, n, hb, step, pre, post, n_plaq);
    if (forms & 2)
        launch_timed(k_tile_rb<T, W, ROWB, false, false, false>, g, b, st, dev_inst, n, hb, step, pre, post, n_plaq);
    return hipGetLastError();
}

int pass_wave_bits(int dtype, int low, int h, int cb)
{
    // low tile of h = 10+W bits, 2 <= W <= 4 (complex64) / 3 (complex128).  High tile with
    // rows of 2^cb amplitudes rotates (6-cb) lane bits + 4 register bits + W wave bits;
    // rows of 128, 256 or 512 bytes (complex64), 128 or 256 bytes (complex128), and for
    // complex128 also 64-byte rows with eight waves: 11 rotated bits in 128 KiB of LDS.
    // Complex128 with 128-byte rows and h = 11 is the register-bit tile (k_tile_rb, eight
    // waves, one more rotated bit in registers).  Either gives a 24-link complex128 step
    // two tile passes (13 + 11 bits) instead of three.
    // Complex128 low tiles of 14 bits are register-bit tiles too (eight waves).
    const int wmax = dtype == LGT_C64 ? 4 : 3;
    if (low && dtype != LGT_C64 && h == 14) return 3;
    if (low) return (h - 10 >= 2 && h - 10 <= wmax) ? h - 10 : -1;
    const int cb_lo = dtype == LGT_C64 ? 4 : 2, cb_hi = dtype == LGT_C64 ? 6 : 4;
    if (cb < cb_lo || cb > cb_hi) return -1;
    if (dtype != LGT_C64 && cb == 3 && h == 11) return 3;
    const int w = h - (10 - cb);
    if (w < 0 || w > wmax) return -1;
    if (dtype != LGT_C64 && cb == 2 && w != 3) return -1;
    return w;
}

bool pass_offsets_fit(int dtype, int n, int low, int hb, int h, int cb)
{
    // per-thread element offsets of a high tile must stay below 2^32 bytes
    const int w = pass_wave_bits(dtype, low, h, cb);
    if (w < 0) return false;
    if (low) return n >= h;
    const int eb = dtype == LGT_C64 ? 3 : 4;
    // half-line rows pair tiles in blocks of 16 (k_tile's tile_of): at least 16 tiles
    if (dtype != LGT_C64 && cb == 2 && n - (10 + w) < 4) return false;
    // the register-bit tile spans 2^(11+w) amplitudes: at least one tile
    if (dtype != LGT_C64 && cb == 3 && h == 11 && n < 11 + w) return false;
    return hb >= cb && hb + h <= n && hb + (6 + w - cb) + eb <= 32;
}

#define LGT_PASS_CASES(T, CB)                                                                   \
    switch (w) {                                                                                \
    case 0: return launch_pass_t<T, 0, CB>(dev_inst, n_inst, n, hb, step, pre, post, n_plaq, forms, merge, st); \
    case 1: return launch_pass_t<T, 1, CB>(dev_inst, n_inst, n, hb, step, pre, post, n_plaq, forms, merge, st); \
    case 2: return launch_pass_t<T, 2, CB>(dev_inst, n_inst, n, hb, step, pre, post, n_plaq, forms, merge, st); \
    case 3: return launch_pass_t<T, 3, CB>(dev_inst, n_inst, n, hb, step, pre, post, n_plaq, forms, merge, st); \
    default: break;                                                                             \
    }

hipError_t launch_tile(int dtype, const DevInst *dev_inst, int n_inst, int n, int low, int hb,
                       int h, int cb, int step, int pre, int post, int n_plaq, int forms,
                       int merge, hipStream_t st)
{
    if (!pass_offsets_fit(dtype, n, low, hb, h, cb)) return hipErrorInvalidValue;
    const int w = pass_wave_bits(dtype, low, h, cb);
    if (dtype == LGT_C64) {
        if (low) {
            if (w == 2) return launch_pass_t<float, 2, 12>(dev_inst, n_inst, n, 0, step, pre, post, n_plaq, forms, merge, st);
            if (w == 3) return launch_pass_t<float, 3, 13>(dev_inst, n_inst, n, 0, step, pre, post, n_plaq, forms, merge, st);
            return launch_pass_t<float, 4, 14>(dev_inst, n_inst, n, 0, step, pre, post, n_plaq, forms, merge, st);
        }
        if (cb == 4) {
            LGT_PASS_CASES(float, 4)
            return launch_pass_t<float, 4, 4>(dev_inst, n_inst, n, hb, step, pre, post, n_plaq, forms, merge, st);
        }
        if (cb == 6) {
            LGT_PASS_CASES(float, 6)
            return launch_pass_t<float, 4, 6>(dev_inst, n_inst, n, hb, step, pre, post, n_plaq, forms, merge, st);
        }
        LGT_PASS_CASES(float, 5)
        return launch_pass_t<float, 4, 5>(dev_inst, n_inst, n, hb, step, pre, post, n_plaq, forms, merge, st);
    }
    if (low) {
        if (h == 14) return launch_pass_rb<double, 3, 13>(dev_inst, n_inst, n, 0, step, pre, post, n_plaq, forms, merge, st);
        if (w == 2) return launch_pass_t<double, 2, 12>(dev_inst, n_inst, n, 0, step, pre, post, n_plaq, forms, merge, st);
        return launch_pass_t<double, 3, 13>(dev_inst, n_inst, n, 0, step, pre, post, n_plaq, forms, merge, st);
    }
    if (cb == 2) {
        if (w == 3) return launch_pass_t<double, 3, 2>(dev_inst, n_inst, n, hb, step, pre, post, n_plaq, forms, merge, st);
    } else if (cb == 3) {
        if (h == 11) return launch_pass_rb<double, 3, 3>(dev_inst, n_inst, n, hb, step, pre, post, n_plaq, forms, merge, st);
        LGT_PASS_CASES(double, 3)
    } else {
        LGT_PASS_CASES(double, 4)
    }
    return hipErrorInvalidValue;
}
#undef LGT_PASS_CASES

template <typename T>
static hipError_t launch_high_t(const DevInst *dev_inst, int n_inst, int n, int q0, int h,
                                int step, int post, int n_plaq, hipStream_t st)
{
    const uint64_t threads = 1ull << (n - h);
    if (threads % kHighThreads) return hipErrorInvalidValue;
    dim3 grid((unsigned)(threads / kHighThreads), (unsigned)n_inst);
    switch (h) {
    case 1: hipLaunchKernelGGL((k_high<T, 1>), grid, dim3(kHighThreads), 0, st, dev_inst, q0, step, post, n_plaq); break;
    case 2: hipLaunchKernelGGL((k_high<T, 2>), grid, dim3(kHighThreads), 0, st, dev_inst, q0, step, post, n_plaq); break;
    case 3: hipLaunchKernelGGL((k_high<T, 3>), grid, dim3(kHighThreads), 0, st, dev_inst, q0, step, post, n_plaq); break;
    case 4: hipLaunchKernelGGL((k_high<T, 4>), grid, dim3(kHighThreads), 0, st, dev_inst, q0, step, post, n_plaq); break;
    case 5: hipLaunchKernelGGL((k_high<T, 5>), grid, dim3(kHighThreads), 0, st, dev_inst, q0, step, post, n_plaq); break;
    case 6: hipLaunchKernelGGL((k_high<T, 6>), grid, dim3(kHighThreads), 0, st, dev_inst, q0, step, post, n_plaq); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_high(int dtype, const DevInst *dev_inst, int n_inst, int n, int q0, int h,
                       int step, int post, int n_plaq, hipStream_t st)
{
    // lanes of a wave must cover 64 consecutive amplitudes: q0 >= 6
    if (q0 < 6 || q0 + h > n || h < 1) return hipErrorInvalidValue;
    if (dtype == LGT_C64) return launch_high_t<float>(dev_inst, n_inst, n, q0, h, step, post, n_plaq, st);
    if (h > 5) return hipErrorInvalidValue;
    return launch_high_t<double>(dev_inst, n_inst, n, q0, h, step, post, n_plaq, st);
}

hipError_t launch_phase(int dtype, const DevInst *dev_inst, int n_inst, int n, int idx,
                        int n_plaq, hipStream_t st)
{
    const uint64_t threads = (1ull << n) >> 4;
    dim3 grid(grid_for(threads > 0 ? threads : 1, 256, 8192), (unsigned)n_inst);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_phase<float>, grid, dim3(256), 0, st, dev_inst, n, idx, n_plaq);
    else
        hipLaunchKernelGGL(k_phase<double>, grid, dim3(256), 0, st, dev_inst, n, idx, n_plaq);
    return hipGetLastError();
}

bool small_supported(int dtype, int n) { (void)dtype; return n >= 6 && n <= 12; }

hipError_t launch_small(int dtype, const DevInst *dev_inst, int n_inst, int n, int n_steps,
                        int pre, int n_plaq, hipStream_t st)
{
    if (!small_supported(dtype, n)) return hipErrorInvalidValue;
    if (n <= 8) {
        // the whole state in one wavefront's registers
#define LGT_WAVE(T, RB) hipLaunchKernelGGL((k_wave<T, RB>), dim3(n_inst), dim3(64), 0, st, dev_inst, n_steps, pre, n_plaq)
        if (dtype == LGT_C64) {
            if (n == 6) LGT_WAVE(float, 0); else if (n == 7) LGT_WAVE(float, 1); else LGT_WAVE(float, 2);
        } else {
            if (n == 6) LGT_WAVE(double, 0); else if (n == 7) LGT_WAVE(double, 1); else LGT_WAVE(double, 2);
        }
#undef LGT_WAVE
        return hipGetLastError();
    }
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_small<float>, dim3(n_inst), dim3(kSmallThreads), 0, st, dev_inst, n,
                           n_steps, pre, n_plaq);
    else
        hipLaunchKernelGGL(k_small<double>, dim3(n_inst), dim3(kSmallThreads), 0, st, dev_inst, n,
                           n_steps, pre, n_plaq);
    return hipGetLastError();
}

hipError_t launch_gate_rx(int dtype, void *psi, int n, int q, double phi, hipStream_t st)
{
    const unsigned g = grid_for(1ull << (n - 1), 256, 16384);
    const double c = std::cos(0.5 * phi), s = std::sin(0.5 * phi);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_gate_rx<float>, dim3(g), dim3(256), 0, st, (float2 *)psi, n, q,
                           (float)c, (float)s);
    else
        hipLaunchKernelGGL(k_gate_rx<double>, dim3(g), dim3(256), 0, st, (double2 *)psi, n, q, c, s);
    return hipGetLastError();
}

hipError_t launch_gate_rz(int dtype, void *psi, int n, int q, double phi, hipStream_t st)
{
    // R_z(phi) = exp(-i sigma^z phi/2): |0> -> e^{-i phi/2}, |1> -> e^{+i phi/2}
    const unsigned g = grid_for(1ull << n, 256, 16384);
    const double c = std::cos(0.5 * phi), s = std::sin(0.5 * phi);
    if (dtype == LGT_C64) {
        float2 e0 = make_float2((float)c, (float)-s), e1 = make_float2((float)c, (float)s);
        hipLaunchKernelGGL(k_gate_rz<float>, dim3(g), dim3(256), 0, st, (float2 *)psi, n, q, e0, e1);
    } else {
        double2 e0 = make_double2(c, -s), e1 = make_double2(c, s);
        hipLaunchKernelGGL(k_gate_rz<double>, dim3(g), dim3(256), 0, st, (double2 *)psi, n, q, e0, e1);
    }
    return hipGetLastError();
}

hipError_t launch_gate_cnot(int dtype, void *psi, int n, int c, int t, hipStream_t st)
{
    if (n < 2 || c == t) return hipErrorInvalidValue;
    const unsigned g = grid_for(1ull << (n - 2), 256, 16384);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_gate_cnot<float>, dim3(g), dim3(256), 0, st, (float2 *)psi, n, c, t);
    else
        hipLaunchKernelGGL(k_gate_cnot<double>, dim3(g), dim3(256), 0, st, (double2 *)psi, n, c, t);
    return hipGetLastError();
}

int reduce_diag_blocks(int n)
{
    const uint64_t work = (1ull << n) / (kRedThreads * 16ull);
    return (int)grid_for(work > 0 ? work : 1, 1, 512);
}

int reduce_blocks(int n)
{
    const uint64_t work = (1ull << n) / (kRedThreads * 16ull);
    return (int)grid_for(work > 0 ? work : 1, 1, 2048);
}

template <typename T>
static void launch_reduce_diag_t(int kb, int g, const void *psi, int n, const uint64_t *masks_dev,
                                 int n_masks, double *partials, hipStream_t st)
{
    using C = cplx_t<T>;
    const C *p = (const C *)psi;
    switch (kb) {
    case 0: hipLaunchKernelGGL((k_red_diag<T, 0>), dim3(g), dim3(kRedThreads), 0, st, p, n, masks_dev, n_masks, partials); break;
    case 1: hipLaunchKernelGGL((k_red_diag<T, 1>), dim3(g), dim3(kRedThreads), 0, st, p, n, masks_dev, n_masks, partials); break;
    case 2: hipLaunchKernelGGL((k_red_diag<T, 2>), dim3(g), dim3(kRedThreads), 0, st, p, n, masks_dev, n_masks, partials); break;
    default: hipLaunchKernelGGL((k_red_diag<T, 3>), dim3(g), dim3(kRedThreads), 0, st, p, n, masks_dev, n_masks, partials); break;
    }
}

hipError_t launch_reduce_diag(int dtype, const void *psi, int n, const uint64_t *masks_dev,
                              int n_masks, double *partials, hipStream_t st)
{
    if (n_masks < 1 || n_masks > kRedMasks || n < 8) return hipErrorInvalidValue;
    // the block count is a power of two (2^(n-12) clamped to [1, 512]); each thread then
    // covers 2^kb amplitudes per outer step, kb <= 3 (8 values: more registers and LDS per
    // thread cost more occupancy than the shorter loop gains; 512 blocks and kb = 3 took
    // 35 us at 24 qubits against 86 us for 2048 blocks and kb = 5)
    const int g = reduce_diag_blocks(n);
    if (g & (g - 1)) return hipErrorInvalidValue;
    const int gb = 31 - __builtin_clz((unsigned)g);
    const int kb = std::min(3, n - 8 - gb);
    if (kb < 0) return hipErrorInvalidValue;
    if (dtype == LGT_C64)
        launch_reduce_diag_t<float>(kb, g, psi, n, masks_dev, n_masks, partials, st);
    else
        launch_reduce_diag_t<double>(kb, g, psi, n, masks_dev, n_masks, partials, st);
    return hipGetLastError();
}

hipError_t launch_reduce_flip(int dtype, const void *psi, int n, const uint64_t *masks_dev,
                              int n_masks, double *partials, hipStream_t st)
{
    if (n_masks < 1 || n_masks > kFlipMasks) return hipErrorInvalidValue;
    const int g = reduce_blocks(n);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_red_flip<float>, dim3(g), dim3(kRedThreads), 0, st,
                           (const float2 *)psi, n, masks_dev, n_masks, partials);
    else
        hipLaunchKernelGGL(k_red_flip<double>, dim3(g), dim3(kRedThreads), 0, st,
                           (const double2 *)psi, n, masks_dev, n_masks, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_dos(int dtype, const void *psi, int n, const uint32_t *ptab_dev,
                             int n_plaq, double *partials, hipStream_t st)
{
    const int g = reduce_blocks(n);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL((k_red_dos<float, false>), dim3(g), dim3(kRedThreads), 0, st,
                           (const float2 *)psi, n, ptab_dev, n_plaq, partials);
    else
        hipLaunchKernelGGL((k_red_dos<double, false>), dim3(g), dim3(kRedThreads), 0, st,
                           (const double2 *)psi, n, ptab_dev, n_plaq, partials);
    return hipGetLastError();
}

hipError_t launch_reduce_popcount(int dtype, const void *psi, int n, const uint32_t *ptab_dev,
                                  double *partials, hipStream_t st)
{
    if (n > kMaxPlaq) return hipErrorInvalidValue;   // bins 0..n must fit the partial width
    const int g = reduce_blocks(n);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL((k_red_dos<float, true>), dim3(g), dim3(kRedThreads), 0, st,
                           (const float2 *)psi, n, ptab_dev, 0, partials);
    else
        hipLaunchKernelGGL((k_red_dos<double, true>), dim3(g), dim3(kRedThreads), 0, st,
                           (const double2 *)psi, n, ptab_dev, 0, partials);
    return hipGetLastError();
}

hipError_t launch_pauli(int dtype, void *psi, int n, uint64_t xmask, uint64_t zmask, hipStream_t st)
{
    if (n < 1 || (xmask >> n) || (zmask >> n)) return hipErrorInvalidValue;
    const unsigned g = grid_for(1ull << n, 256, 16384);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_pauli<float>, dim3(g), dim3(256), 0, st, (float2 *)psi, n, xmask, zmask);
    else
        hipLaunchKernelGGL(k_pauli<double>, dim3(g), dim3(256), 0, st, (double2 *)psi, n, xmask, zmask);
    return hipGetLastError();
}

hipError_t launch_gate_h(int dtype, void *psi, int n, int q, hipStream_t st)
{
    const uint64_t half = 1ull << (n - 1);
    const unsigned g = grid_for(half, 256, 16384);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_gate_h<float>, dim3(g), dim3(256), 0, st, (float2 *)psi, n, q);
    else
        hipLaunchKernelGGL(k_gate_h<double>, dim3(g), dim3(256), 0, st, (double2 *)psi, n, q);
    return hipGetLastError();
}

hipError_t launch_gate_cz(int dtype, void *psi, int n, int a, int b, hipStream_t st)
{
    if (a == b || a < 0 || b < 0 || a >= n || b >= n) return hipErrorInvalidValue;
    const unsigned g = grid_for(1ull << n, 256, 16384);
    const uint64_t both = (1ull << a) | (1ull << b);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_gate_cz<float>, dim3(g), dim3(256), 0, st, (float2 *)psi, n, both);
    else
        hipLaunchKernelGGL(k_gate_cz<double>, dim3(g), dim3(256), 0, st, (double2 *)psi, n, both);
    return hipGetLastError();
}

hipError_t launch_project_scale(int dtype, void *psi, int n, uint64_t zero_mask, double scale,
                                hipStream_t st)
{
    const unsigned g = grid_for(1ull << n, 256, 16384);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_project_scale<float>, dim3(g), dim3(256), 0, st, (float2 *)psi, n,
                           zero_mask, (float)scale);
    else
        hipLaunchKernelGGL(k_project_scale<double>, dim3(g), dim3(256), 0, st, (double2 *)psi, n,
                           zero_mask, scale);
    return hipGetLastError();
}

hipError_t launch_sum_cols(const double *partials, int rows, int width, int ncols, double *out,
                           hipStream_t st)
{
    if (rows < 1 || ncols < 1 || ncols > width) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sum_cols, dim3(ncols), dim3(kRedThreads), 0, st, partials, rows, width, out);
    return hipGetLastError();
}

int sample_block_bits(int n) { return n < kSampleBlockBits ? n : kSampleBlockBits; }

hipError_t launch_sample_scratch(int dtype, const void *psi, int n, uint64_t n_shots,
                                 uint64_t seed, void *scratch_dev, hipStream_t st)
{
    const uint64_t nb = 1ull << (n - sample_block_bits(n));
    if (nb > (uint64_t)kScratchSums || n_shots < 1 || n_shots > (uint64_t)kScratchShots)
        return hipErrorInvalidValue;
    double *sums = (double *)scratch_dev;
    uint64_t *shots = (uint64_t *)scratch_dev + kScratchSums;
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_block_sums<float>, dim3((unsigned)nb), dim3(256), 0, st,
                           (const float2 *)psi, n, sums);
    else
        hipLaunchKernelGGL(k_block_sums<double>, dim3((unsigned)nb), dim3(256), 0, st,
                           (const double2 *)psi, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_prefix_seq, dim3(1), dim3(64), 0, st, sums, (int)nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const unsigned g = (unsigned)((n_shots + 255) / 256);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_sample<float>, dim3(g), dim3(256), 0, st, (const float2 *)psi, n,
                           sums, (int)nb, n_shots, seed, shots);
    else
        hipLaunchKernelGGL(k_sample<double>, dim3(g), dim3(256), 0, st, (const double2 *)psi, n,
                           sums, (int)nb, n_shots, seed, shots);
    return hipGetLastError();
}

hipError_t launch_sample(int dtype, const void *psi, int n, uint64_t n_shots, uint64_t seed,
                         double *block_sums, double *block_prefix, uint64_t *out_dev,
                         hipStream_t st)
{
    const int nb = 1 << (n - sample_block_bits(n));
    hipError_t e;
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_block_sums<float>, dim3(nb), dim3(256), 0, st, (const float2 *)psi,
                           n, block_sums);
    else
        hipLaunchKernelGGL(k_block_sums<double>, dim3(nb), dim3(256), 0, st,
                           (const double2 *)psi, n, block_sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // inclusive prefix on the host in FP64, ascending block order
    std::vector<double> h(nb);
    if ((e = hipMemcpyAsync(h.data(), block_sums, sizeof(double) * nb, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    double acc = 0;
    for (int i = 0; i < nb; ++i) {
        acc += h[i];
        h[i] = acc;
    }
    if ((e = hipMemcpyAsync(block_prefix, h.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    const unsigned g = (unsigned)((n_shots + 255) / 256);
    if (dtype == LGT_C64)
        hipLaunchKernelGGL(k_sample<float>, dim3(g), dim3(256), 0, st, (const float2 *)psi, n,
                           block_prefix, nb, n_shots, seed, out_dev);
    else
        hipLaunchKernelGGL(k_sample<double>, dim3(g), dim3(256), 0, st, (const double2 *)psi, n,
                           block_prefix, nb, n_shots, seed, out_dev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

}  // namespace lgt
