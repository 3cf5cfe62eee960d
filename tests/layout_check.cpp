// Host check of the tile-pass layouts (tile_layout.hpp) for every geometry the library
// instantiates.  For each (element type, waves W, row bits ROWB):
//  * layout B is a bijection of the tile bits (lanes, waves, registers);
//  * each rotation round (before and after the phase) rotates every tile bit at or above
//    the row bits exactly once, and only lane bits 0..3 are rotated across lanes;
//  * the LDS slot of an element is the same in both layouts' formulas (additive in the
//    register offset), the slots of the whole tile are a bijection, and every 16 lanes of
//    one LDS access hit 16 distinct values of the low four slot bits.
// Prints one line per geometry and returns non-zero on any failure.
#include <cstdio>

#include "tile_layout.hpp"

using namespace lgt;

template <typename T, int W, int ROWB>
int check()
{
    using PG = PassGeom<T, W, ROWB>;
    using MG = MergeGeom<T, W, ROWB>;
    constexpr int TB = PG::TB, CB = PG::LOW ? 0 : PG::CB;
    constexpr MergeLayout M = MG::M;
    int bad = 0;
    int seen = 0;
    for (int k = 0; k < 6; ++k) seen |= 1 << M.lane[k];
    for (int k = 0; k < W; ++k) seen |= 1 << M.wave[k];
    for (int k = 0; k < 4; ++k) seen |= 1 << M.reg[k];
    if (seen != (1 << TB) - 1 || __builtin_popcount(seen) != 10 + W) {
        std::printf("  layout B is not a bijection of the tile bits (%x)\n", seen);
        ++bad;
    }
    // rotated bits of the two rounds: A registers and A lanes 0..3, B registers and B lanes
    auto regA = [](int k) { return 6 + W + k; };
    int r1 = 0, r2 = 0, dup = 0;
    auto add = [&](int &acc, int b) {
        if (acc & (1 << b)) ++dup;
        acc |= 1 << b;
    };
    for (int k = 0; k < 4; ++k) add(r1, regA(k));
    for (int k = 0; k < 4; ++k)
        if (M.al & (1 << k)) add(r1, k);
    for (int k = 0; k < 4; ++k)
        if (M.br1 & (1 << k)) add(r1, M.reg[k]);
    for (int k = 0; k < 6; ++k)
        if (M.bl & (1 << k)) {
            add(r1, M.lane[k]);
            if (k > 3) ++dup;   // cross-row lane rotations are not allowed
        }
    for (int k = 0; k < 4; ++k) add(r2, M.reg[k]);
    for (int k = 0; k < 6; ++k)
        if (M.bl & (1 << k)) add(r2, M.lane[k]);
    for (int k = 0; k < 4; ++k)
        if (M.ar2 & (1 << k)) add(r2, regA(k));
    for (int k = 0; k < 4; ++k)
        if (M.al & (1 << k)) add(r2, k);
    const int rot = ((1 << TB) - 1) & ~((1 << CB) - 1);
    if (r1 != rot || r2 != rot || dup) {
        std::printf("  rotation cover r1=%x r2=%x want=%x dup=%d\n", r1, r2, rot, dup);
        ++bad;
    }
    static int hitA[1 << 14], hitB[1 << 14];
    for (int i = 0; i < (1 << TB); ++i) hitA[i] = hitB[i] = 0;
    for (int w = 0; w < (1 << W); ++w)
        for (int l = 0; l < 64; ++l) {
            const int oA = l | (w << 6), oB = MG::thrB(l, w);
            for (int r = 0; r < 16; ++r) {
                const int sa = MG::swz(oA) + (r << (6 + W)), sb = MG::swz(oB) + MG::regB(r);
                if (sa != MG::swz(oA | (r << (6 + W))) || sb != MG::swz(oB | MG::regB(r))) {
                    std::printf("  slot formula not additive\n");
                    return bad + 1;
                }
                if (sa < 0 || sa >= (1 << TB) || sb < 0 || sb >= (1 << TB)) {
                    std::printf("  slot out of range\n");
                    return bad + 1;
                }
                hitA[sa]++;
                hitB[sb]++;
            }
        }
    for (int i = 0; i < (1 << TB); ++i)
        if (hitA[i] != 1 || hitB[i] != 1) {
            std::printf("  slot %d written %d / read %d times\n", i, hitA[i], hitB[i]);
            ++bad;
            break;
        }
    for (int w = 0; w < (1 << W); ++w)
        for (int g = 0; g < 4; ++g)
            for (int r = 0; r < 16; ++r) {
                int mA = 0, mB = 0;
                for (int l = 16 * g; l < 16 * g + 16; ++l) {
                    mA |= 1 << ((MG::swz(l | (w << 6)) + (r << (6 + W))) & 15);
                    mB |= 1 << ((MG::swz(MG::thrB(l, w)) + MG::regB(r)) & 15);
                }
                if (mA != 0xFFFF || mB != 0xFFFF) {
                    std::printf("  LDS bank groups A %x B %x\n", mA, mB);
                    return bad + 1;
                }
            }
    std::printf("%s W=%d ROWB=%d tile bits %d row bits %d: %s\n", sizeof(T) == 4 ? "c64" : "c128",
                W, ROWB, TB, CB, bad ? "BAD" : "ok");
    return bad;
}

int main()
{
    int bad = 0;
    // low tiles
    bad += check<float, 2, 12>() + check<float, 3, 13>() + check<float, 4, 14>();
    bad += check<double, 2, 12>() + check<double, 3, 13>();
    // high tiles: complex64 rows of 16, 32 or 64 amplitudes, complex128 rows of 4 (only with 8 waves), 8 or 16
    bad += check<float, 0, 4>() + check<float, 1, 4>() + check<float, 2, 4>() + check<float, 3, 4>() + check<float, 4, 4>();
    bad += check<float, 0, 5>() + check<float, 1, 5>() + check<float, 2, 5>() + check<float, 3, 5>() + check<float, 4, 5>();
    bad += check<float, 0, 6>() + check<float, 1, 6>() + check<float, 2, 6>() + check<float, 3, 6>() + check<float, 4, 6>();
    bad += check<double, 3, 2>();
    bad += check<double, 0, 3>() + check<double, 1, 3>() + check<double, 2, 3>() + check<double, 3, 3>();
    bad += check<double, 0, 4>() + check<double, 1, 4>() + check<double, 2, 4>() + check<double, 3, 4>();
    std::printf("failures: %d\n", bad);
    return bad != 0;
}
