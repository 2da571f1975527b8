// Host check of the shell slot layout of the pushed moments (the library's
// own Shell<TX, TY, ZC>): for every tile chunk extent W <= TX, H <= TY,
// Zc <= ZC, the targets a chunk writes to its shell (the tile + 1 ring of each
// of its planes, the whole tile + 1 face below and above) get distinct slots
// inside [0, SIZE); and the XCD order of the tile launches (check_xcd).
// Built and run by test_shell_layout.py; exit status 0 on success.
#include <cstdio>
#include <vector>

#include "lbm_kernels.hpp"

template <int TX, int TY, int ZC>
static int check()
{
    using SH = evlbm::Shell<TX, TY, ZC>;
    // every moment and chunk starts on a 128-byte line (32 FP32 values), and
    // so does every ring row of a 32- or 64-wide tile
    for (int lz = 0; lz < ZC; ++lz)
        if (SH::SIZE % 32 != 0 ||
            (TX % 32 == 0 && (SH::slot(0, -1, lz, TX, TY, ZC) % 32 != 0 || SH::slot(0, TY, lz, TX, TY, ZC) % 32 != 0))) {
            std::printf("TX %d TY %d ZC %d: SIZE %d or a ring row of plane %d is not line-aligned\n", TX, TY, ZC,
                        SH::SIZE, lz);
            return 1;
        }
    long cases = 0;
    for (int W = 1; W <= TX; ++W)
        for (int H = 1; H <= TY; ++H)
            for (int Zc = 1; Zc <= ZC; ++Zc) {
                std::vector<int> seen(SH::SIZE, 0);
                auto put = [&](int lx, int ly, int lz) {
                    const int s = SH::slot(lx, ly, lz, W, H, Zc);
                    if (s < 0 || s >= SH::SIZE || seen[s]++) {
                        std::printf("TX %d TY %d ZC %d: W %d H %d Zc %d target (%d, %d, %d) slot %d %s\n", TX, TY, ZC,
                                    W, H, Zc, lx, ly, lz, s, (s < 0 || s >= SH::SIZE) ? "out of range" : "reused");
                        return false;
                    }
                    return true;
                };
                for (int lz = -1; lz <= Zc; ++lz)
                    for (int ly = -1; ly <= H; ++ly)
                        for (int lx = -1; lx <= W; ++lx) {
                            const bool inside = lx >= 0 && lx < W && ly >= 0 && ly < H && lz >= 0 && lz < Zc;
                            if (!inside && !put(lx, ly, lz)) return 1;
                        }
                ++cases;
            }
    std::printf("Shell<%d, %d, %d>: %ld chunk extents, slots distinct and in range\n", TX, TY, ZC, cases);
    return 0;
}

// The XCD order of the tile launches (xcd_tile): for T tiles per chunk and
// nchunk chunks, the map of block indices onto tiles is a bijection of
// [0, T nchunk) (no tile skipped or run twice), and when 8 divides T the
// blocks of one XCD (equal b mod 8) take one contiguous run of every chunk.
static int check_xcd()
{
    for (int T = 1; T <= 1100; ++T)
        for (int nchunk : {1, 3, 7}) {
            const int n = T * nchunk;
            std::vector<int> seen(n, 0);
            for (int b = 0; b < n; ++b) {
                const int t = evlbm::xcd_tile(b, T);
                if (t < 0 || t >= n || seen[t]++) {
                    std::printf("xcd_tile: T %d, %d chunks: block %d -> tile %d out of range or repeated\n", T,
                                nchunk, b, t);
                    return 1;
                }
            }
            if (T % 8) continue;
            for (int c = 0; c < nchunk; ++c)
                for (int j = 0; j < 8; ++j) {
                    int lo = n, hi = -1, count = 0;
                    for (int b = 0; b < n; ++b) {
                        const int t = evlbm::xcd_tile(b, T);
                        if ((b & 7) == j && t / T == c) {
                            lo = t < lo ? t : lo;
                            hi = t > hi ? t : hi;
                            ++count;
                        }
                    }
                    if (count != T / 8 || hi - lo + 1 != count) {
                        std::printf("xcd_tile: T %d, chunk %d, XCD %d: tiles not one contiguous run of %d\n", T, c,
                                    j, T / 8);
                        return 1;
                    }
                }
        }
    return 0;
}

int main()
{
    return check<64, 4, 40>() | check<16, 8, 64>() | check<16, 8, 40>() | check<64, 4, 32>() | check_xcd();
}
