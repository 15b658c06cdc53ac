// Host build of the library's block-space maps (the same inline header the
// kernels use), for running under AddressSanitizer and UndefinedBehaviorSanitizer:
// every block of every map is decoded for a range of nb, and the mapped tiles
// must cover the target simplex exactly once (and the lambda inverses must
// return each block), with no shift, overflow or out-of-range access.  The
// column-major and patch enumerations of Pi2 and the XCD renumbering must be
// permutations of their ranges.  Exit status 0 and "ok" on success.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "smx_maps.h"
#include "smx_maps_inv.h"

using namespace smx;

static long long binom(long long n, int k) {
    long long v = 1;
    for (int i = 0; i < k; ++i) v = v * (n - i) / (i + 1);
    return v;
}

// rank of a sorted tuple in [0, nb)^m (colex), for the visited bitmap
static long long rank_tuple(const int *t, int m) {
    long long r = 0;
    for (int d = 0; d < m; ++d) r += binom(t[d] + d, d + 1);
    return r;
}

static int fails = 0;

static void check(int m, int nb, int map) {
    const int lg = ceil_log2_u64(uint64_t(nb));
    uint64_t G = 0;
    uint32_t main = 0;
    if (map == MAP_LAMBDA) {
        if (m == 2) G = lambda2_blocks(lg);
        if (m == 3) { main = lambda3_main_blocks(lg); G = main + lambda2_blocks(lg); }
        if (m == 4) { main = uint32_t(lambda4_main_blocks(lg)); G = main + lambda3_main_blocks(lg) + lambda2_blocks(lg); }
    } else if (map == MAP_REC) {
        G = rec_blocks(m, lg);
    } else if (map == MAP_BELOW) {
        G = m == 2 ? below2_blocks(uint64_t(nb)) : below3_blocks(uint64_t(nb));
    } else {  // linear
        G = uint64_t(binom(nb + m - 1, m));
    }
    const long long target = binom(nb + m - 1, m);
    std::vector<unsigned char> seen(size_t(target), 0);
    long long mapped = 0;
    for (uint64_t id = 0; id < G; ++id) {
        int t[4] = {0, 0, 0, 0};
        bool ok = false;
        if (m == 2) {
            if (map == MAP_LAMBDA) ok = lambda2(uint32_t(id), lg, nb, t[0], t[1]);
            else if (map == MAP_REC) ok = rec2(uint32_t(id), lg, nb, uint32_t(G), t[0], t[1]);
            else if (map == MAP_BELOW) ok = below2(id, uint32_t(nb), t[0], t[1]);
            else { linear2(uint32_t(id), t[0], t[1]); ok = true; }
        } else if (m == 3) {
            if (map == MAP_LAMBDA) ok = lambda3(uint32_t(id), lg, nb, main, t[0], t[1], t[2]);
            else if (map == MAP_REC) ok = rec3(uint32_t(id), lg, nb, uint32_t(G), t[0], t[1], t[2]);
            else if (map == MAP_BELOW) ok = below3(id, uint32_t(nb), t[0], t[1], t[2]);
            else { linear3(uint32_t(id), t[0], t[1], t[2]); ok = true; }
        } else {
            if (map == MAP_LAMBDA) ok = lambda4(uint32_t(id), lg, nb, main, t);
            else if (map == MAP_REC) ok = rec4(uint32_t(id), lg, nb, uint32_t(G), t);
            else { linear4(uint32_t(id), t); ok = true; }
        }
        if (!ok) continue;
        for (int d = 0; d < m; ++d) {
            const bool bad = t[d] < 0 || t[d] >= nb || (d > 0 && t[d] < t[d - 1]);
            if (bad) {
                if (fails++ < 10) std::printf("m=%d nb=%d map=%d block %llu: tile out of the simplex\n", m, nb, map,
                                              (unsigned long long)id);
                ok = false;
                break;
            }
        }
        if (!ok) continue;
        if (map == MAP_LAMBDA && m <= 3) {  // the inverse map returns this block
            const uint64_t back = m == 2 ? lambda2_inv(lg, uint32_t(t[0]), uint32_t(t[1]))
                                         : lambda3_inv(lg, main, uint32_t(t[0]), uint32_t(t[1]), uint32_t(t[2]));
            if (back != id && fails++ < 10)
                std::printf("m=%d nb=%d: inverse of block %llu gave %llu\n", m, nb, (unsigned long long)id,
                            (unsigned long long)back);
        }
        const long long r = rank_tuple(t, m);
        if (seen[size_t(r)]++) {
            if (fails++ < 10) std::printf("m=%d nb=%d map=%d: tile mapped twice\n", m, nb, map);
        }
        ++mapped;
    }
    if (mapped != target && fails++ < 10)
        std::printf("m=%d nb=%d map=%d: %lld of %lld tiles mapped\n", m, nb, map, mapped, target);
}

// lambda2 through the column-major enumeration of Pi2, after the XCD
// renumbering (the Gram kernel's composition): each id in [0, G) reaches a
// distinct Pi2 point, and the mapped tiles cover the nb(nb+1)/2 tiles once.
static void check_cm(int nb) {
    const int lg = ceil_log2_u64(uint64_t(nb));
    const uint32_t G = lambda2_blocks(lg);
    std::vector<unsigned char> hit(G, 0), seen(size_t(binom(nb + 1, 2)), 0);
    long long mapped = 0;
    for (uint32_t id = 0; id < G; ++id) {
        const uint32_t r = xcd_remap(id, G);
        const uint32_t xf = r < G ? lambda2_cm_to_xfast(r, lg) : G;
        if (xf >= G || hit[xf]++) {
            if (fails++ < 10) std::printf("cm nb=%d: id %u is not a permutation\n", nb, id);
            continue;
        }
        int x = 0, y = 0;
        if (!lambda2_cm(r, lg, nb, x, y)) continue;
        if (x < 0 || y < x || y >= nb) {
            if (fails++ < 10) std::printf("cm nb=%d: id %u tile out of the simplex\n", nb, id);
            continue;
        }
        const int t[2] = {x, y};
        if (seen[size_t(rank_tuple(t, 2))]++ && fails++ < 10) std::printf("cm nb=%d: tile mapped twice\n", nb);
        ++mapped;
    }
    if (mapped != binom(nb + 1, 2) && fails++ < 10) std::printf("cm nb=%d: %lld tiles mapped\n", nb, mapped);
}

// the patch enumeration of Pi2 is a permutation of its ids for every patch shape
static void check_patch(int lg) {
    const uint32_t G = lambda2_blocks(lg);
    for (int pxl = 0; pxl <= 6; ++pxl)
        for (int pyl = 0; pyl <= 6; ++pyl) {
            std::vector<unsigned char> hit(G, 0);
            for (uint32_t id = 0; id < G; ++id) {
                const uint32_t xf = lambda2_patch_to_xfast(id, lg, pxl, pyl);
                if ((xf >= G || hit[xf]++) && fails++ < 10)
                    std::printf("patch lg=%d %dx%d: id %u -> %u\n", lg, pxl, pyl, id, xf);
            }
        }
}

// the XCD renumbering is a bijection on [0, G) for every G, including G < 8
static void check_xcd(uint32_t G) {
    std::vector<unsigned char> hit(G, 0);
    for (uint32_t b = 0; b < G; ++b) {
        const uint32_t r = xcd_remap(b, G);
        if ((r >= G || hit[r]++) && fails++ < 10) std::printf("xcd G=%u: %u -> %u\n", G, b, r);
    }
}

int main() {
    for (int nb = 1; nb <= 300; nb += (nb < 40 ? 1 : 37)) check_cm(nb);
    for (uint32_t G = 1; G <= 200; ++G) check_xcd(G);
    for (int lg = 0; lg <= 10; ++lg) check_patch(lg);
    check_xcd(8191u * 4097u);
    const int maps2[] = {MAP_LAMBDA, MAP_LINEAR, MAP_BELOW, MAP_REC};
    for (int nb = 1; nb <= 300; nb += (nb < 40 ? 1 : 37))
        for (int map : maps2) check(2, nb, map);
    for (int nb = 1; nb <= 80; nb += (nb < 24 ? 1 : 13))
        for (int map : maps2) check(3, nb, map);
    const int maps4[] = {MAP_LAMBDA, MAP_LINEAR, MAP_REC};
    for (int nb = 1; nb <= 40; nb += (nb < 12 ? 1 : 9))
        for (int map : maps4) check(4, nb, map);
    if (fails) {
        std::printf("%d failures\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
