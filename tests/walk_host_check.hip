// Host build of the culling walk (Section 3.2) checked against the oracle's
// plain voxel-by-voxel walk: random clustered blocker fields, random start
// voxels and eyes (anywhere, on voxel-centre ties, inside the grid, far away)
// and blocking limits 1, 4 and unbounded.  The cell flags here are computed
// from the blocker field directly.  Prints "checks=N bad=M"; exit status 1 on
// any mismatch.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "vrt_cullwalk.h"

extern "C" int64_t orc_culling_ray(int64_t x, int64_t y, int64_t z, const int64_t *E, const int32_t *G,
                                   const uint8_t *blocking, int64_t limit, int64_t *n_visited);

namespace {

// Blocker flags of every cell size the walk asks about, from the voxel field.
struct HostCells {
    int G[3];
    const uint8_t *blk;
    std::vector<uint8_t> flag[7];  // flag[s]: cells of 2^s voxels a side holding a blocker
    int n[7][3];

    void build() {
        for (int s = 1; s <= 6; ++s) {
            for (int a = 0; a < 3; ++a) n[s][a] = (G[a] + (1 << s) - 1) >> s;
            flag[s].assign((size_t)n[s][0] * n[s][1] * n[s][2], 0);
        }
        for (int z = 0; z < G[2]; ++z)
            for (int y = 0; y < G[1]; ++y)
                for (int x = 0; x < G[0]; ++x)
                    if (blocking(x, y, z))
                        for (int s = 1; s <= 6; ++s) flag[s][idx(s, x, y, z)] = 1;
    }
    size_t idx(int s, int x, int y, int z) const {
        return ((size_t)(z >> s) * n[s][1] + (y >> s)) * n[s][0] + (x >> s);
    }
    bool blocking(int x, int y, int z) const { return blk[((size_t)z * G[1] + y) * G[0] + x] != 0; }
    bool brick_empty(int x, int y, int z) const { return !flag[3][idx(3, x, y, z)]; }
    int empty_shift(int x, int y, int z) const {
        if (!flag[6][idx(6, x, y, z)]) return 6;
        if (!flag[5][idx(5, x, y, z)]) return 5;
        if (!flag[4][idx(4, x, y, z)]) return 4;
        return 3;
    }
    uint64_t slice_bits(int x, int y, int z) const {  // blocking voxels of the brick's z-slice, bit 8 y + x
        uint64_t m = 0;
        for (int Y = 0; Y < 8; ++Y)
            for (int X = 0; X < 8; ++X) {
                const int cx = (x & ~7) + X, cy = (y & ~7) + Y;
                if (cx < G[0] && cy < G[1] && blocking(cx, cy, z)) m |= 1ull << (8 * Y + X);
            }
        return m;
    }
    uint64_t sub_mask(int x, int y, int z) const {  // 2^3 cells of the brick, bit 16 Z + 4 Y + X
        uint64_t m = 0;
        for (int Z = 0; Z < 4; ++Z)
            for (int Y = 0; Y < 4; ++Y)
                for (int X = 0; X < 4; ++X) {
                    const int cx = (x & ~7) + 2 * X, cy = (y & ~7) + 2 * Y, cz = (z & ~7) + 2 * Z;
                    if (cx < G[0] && cy < G[1] && cz < G[2] && flag[1][idx(1, cx, cy, cz)])
                        m |= 1ull << (16 * Z + 4 * Y + X);
                }
        return m;
    }
};

}  // namespace

int main(int argc, char **argv) {
    std::mt19937_64 rng(argc > 1 ? strtoull(argv[1], nullptr, 10) : 1);
    const int per_field = argc > 2 ? atoi(argv[2]) : 4000;
    const int dims[][3] = {{40, 48, 56}, {128, 128, 128}, {200, 72, 136}, {8, 8, 8}};
    long checks = 0, bad = 0;
    for (const auto &d : dims) {
        for (int field = 0; field < 6; ++field) {
            int G[3] = {d[0], d[1], d[2]};
            std::vector<uint8_t> blk((size_t)G[0] * G[1] * G[2], 0);
            if (field < 5) {  // a few boxes, three quarters of their voxels blocking
                const int nbox = 1 + (int)(rng() % 6);
                for (int b = 0; b < nbox; ++b) {
                    int lo[3], hi[3];
                    for (int a = 0; a < 3; ++a) {
                        lo[a] = (int)(rng() % G[a]);
                        hi[a] = std::min(G[a], lo[a] + 1 + (int)(rng() % 12));
                    }
                    for (int z = lo[2]; z < hi[2]; ++z)
                        for (int y = lo[1]; y < hi[1]; ++y)
                            for (int x = lo[0]; x < hi[0]; ++x)
                                if (rng() % 4) blk[((size_t)z * G[1] + y) * G[0] + x] = 1;
                }
            }
            HostCells C;
            for (int a = 0; a < 3; ++a) C.G[a] = G[a];
            C.blk = blk.data();
            C.build();
            int bbox[6] = {1 << 30, 1 << 30, 1 << 30, -(1 << 30), -(1 << 30), -(1 << 30)};
            for (int z = 0; z < G[2]; ++z)
                for (int y = 0; y < G[1]; ++y)
                    for (int x = 0; x < G[0]; ++x)
                        if (C.blocking(x, y, z)) {
                            bbox[0] = std::min(bbox[0], x), bbox[1] = std::min(bbox[1], y), bbox[2] = std::min(bbox[2], z);
                            bbox[3] = std::max(bbox[3], x), bbox[4] = std::max(bbox[4], y), bbox[5] = std::max(bbox[5], z);
                        }
            for (int r = 0; r < per_field; ++r) {
                int v[3];
                for (int a = 0; a < 3; ++a) v[a] = (int)(rng() % G[a]);
                int64_t E[3];
                const int kind = (int)(rng() % 4);
                for (int a = 0; a < 3; ++a) {
                    const long long c = (long long)v[a] * 256 + 128;
                    if (kind == 0) E[a] = (long long)(rng() % (6ull * G[a] * 256)) - 3ll * G[a] * 256;
                    else if (kind == 1) E[a] = c + ((long long)(rng() % 9) - 4) * 128 * (long long)(1 + rng() % 40);
                    else if (kind == 2) E[a] = (long long)(rng() % ((unsigned long long)G[a] * 256));
                    else E[a] = ((rng() % 2) ? 1 : -1) * (long long)(rng() % 4000000);
                }
                const int limit = r % 3 == 0 ? 1 : (r % 3 == 1 ? 4 : 100000);
                const long long El[3] = {E[0], E[1], E[2]};
                const int got = vrt::culling_walk(G, v[0], v[1], v[2], El, limit, bbox, C);
                int64_t visited;
                const int64_t want = orc_culling_ray(v[0], v[1], v[2], E, G, blk.data(), limit, &visited);
                ++checks;
                if (got != want) {
                    if (bad < 10)
                        printf("mismatch G=%d,%d,%d v=%d,%d,%d E=%lld,%lld,%lld limit=%d walk=%d oracle=%lld\n", G[0],
                               G[1], G[2], v[0], v[1], v[2], (long long)E[0], (long long)E[1], (long long)E[2], limit,
                               got, (long long)want);
                    ++bad;
                }
            }
        }
    }
    printf("checks=%ld bad=%ld\n", checks, bad);
    return bad != 0;
}
