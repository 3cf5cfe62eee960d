// Register and LDS layouts of the tile passes (k_tile in kernels.hip), as compile-time
// functions only: no HIP types, so the same definitions compile for the device and for a
// host-side check of every geometry (coverage of the rotated bits, slot bijection, LDS
// banks).
#pragma once

namespace lgt {

template <typename T, int W, int ROWB>
struct PassGeom {
    static constexpr bool LOW = ROWB >= 10 + W;
    static constexpr int TB = 10 + W;                        // tile bits
    static constexpr int CB = LOW ? TB : ROWB;               // contiguous row bits
};

// ---------------------------------------------------------------------------
// Tile pass k_tile.  Each tile goes through two register layouts and back:
//   layout A (load and store): tile bit 0..5 = lane, 6..5+W = wave, 6+W..9+W = register;
//   layout B (after one LDS exchange): chosen so that every rotated bit is a register
//   bit or one of the lane bits 0..3 (DPP within a row of 16) in A or in B.
// A rotates its register bits and its lane bits 0..3; B rotates A's wave bits and tile
// bits 4, 5 (in registers, at most two on DPP lanes).  The phase is applied in B, then
// the tile goes back to A for the store.  A merged launch (MERGE) also applies the
// next step's rotations after the phase: first B's, then A's, so every bit is rotated
// once per step and in the same order in every kind of launch.  No bit needs a lane
// exchange across rows.  In each exchange a thread writes exactly the LDS slots it read
// in the previous one, so only the barrier between a write and the matching read is
// needed (two per tile).  An XOR of tile bits 4, 5 into slot bits 2, 3 keeps every LDS
// access of 16 lanes on 16 distinct consecutive slots.
// ---------------------------------------------------------------------------
struct MergeLayout {
    int lane[6], wave[4], reg[4];   // tile bit of each B lane, wave and register index bit
    int br1;                        // B register bits rotated before the phase
    int bl;                         // B lane bits rotated across lanes (both rounds)
    int al;                         // A lane bits rotated across lanes (both rounds)
    int ar2;                        // A register bits rotated after the phase
    int n_swz, swz_src[2], swz_dst[2];
};

constexpr MergeLayout merge_layout(int W, int TB, int CB)
{
    MergeLayout m{};
    bool used[16] = {};
    int need[6] = {}, nn = 0;
    for (int k = 0; k < W; ++k) need[nn++] = 6 + k;          // A's wave bits
    for (int b = 5; b >= 4; --b)
        if (b >= CB) need[nn++] = b;                          // rotated lane bits 4, 5
    int nr = 0;
    for (int i = 0; i < nn && nr < 4; ++i) {
        m.reg[nr++] = need[i];
        used[need[i]] = true;
    }
    m.br1 = (1 << nr) - 1;
    for (int k = 0; nr < 4; ++k) {                            // fillers: A register bits
        m.reg[nr++] = 6 + W + k;
        used[6 + W + k] = true;
    }
    int nl = 0;
    for (int i = 4; i < nn; ++i) {                            // the rest of `need` on DPP lanes
        m.lane[nl++] = need[i];
        used[need[i]] = true;
    }
    m.bl = (1 << nl) - 1;
    for (int b = 0; b < TB && nl < 6; ++b)
        if (!used[b]) {
            m.lane[nl++] = b;
            used[b] = true;
        }
    int nw = 0;
    for (int b = 0; b < TB; ++b)
        if (!used[b]) m.wave[nw++] = b;
    m.al = 0;
    for (int k = CB; k < 4; ++k) m.al |= 1 << k;
    m.ar2 = 15;
    for (int k = 0; k < 4; ++k)
        if (m.reg[k] >= 6 + W) m.ar2 &= ~(1 << (m.reg[k] - 6 - W));
    // tile bits >= 4 on B lanes 0..3 pair with the bits of 0..3 missing there
    bool in_lo[4] = {};
    int ext[4] = {}, ne = 0;
    for (int k = 0; k < 4; ++k) {
        if (m.lane[k] < 4) in_lo[m.lane[k]] = true;
        else ext[ne++] = m.lane[k];
    }
    for (int b = 0, i = 0; b < 4 && i < ne; ++b)
        if (!in_lo[b]) {
            m.swz_src[i] = ext[i];
            m.swz_dst[i] = b;
            ++i;
            m.n_swz = i;
        }
    return m;
}

template <typename T, int W, int ROWB>
struct MergeGeom {
    using PG = PassGeom<T, W, ROWB>;
    static constexpr int TB = PG::TB, CB = PG::CB;
    static constexpr MergeLayout M = merge_layout(W, TB, PG::LOW ? 0 : CB);
    // tile offset of B register index r
    static constexpr int regB(int r)
    {
        int o = 0;
        for (int k = 0; k < 4; ++k)
            if (r & (1 << k)) o |= 1 << M.reg[k];
        return o;
    }
    static constexpr int swz(int o)
    {
        for (int i = 0; i < M.n_swz; ++i) o ^= ((o >> M.swz_src[i]) & 1) << M.swz_dst[i];
        return o;
    }
    // tile offset of B lane l, wave w, register 0
    static constexpr int thrB(int l, int w)
    {
        int o = 0;
        for (int k = 0; k < 6; ++k) o |= ((l >> k) & 1) << M.lane[k];
        for (int k = 0; k < W; ++k) o |= ((w >> k) & 1) << M.wave[k];
        return o;
    }
};

}  // namespace lgt
