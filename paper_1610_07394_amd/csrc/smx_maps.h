// Block-space maps from a launched block to a simplex tile.
//
// Every function here is block-uniform: it depends only on the block index,
// so on gfx950 the integer work runs on the scalar unit (s_flbit for clz,
// s_lshl / s_lshr for powers of two) and costs no vector ALU slots.  The same
// inline code is compiled for the host so the host-side query can evaluate it.
//
// Tile targets: T2 = {X <= Y < nb}, T3 = {X <= Y <= Z < nb},
// T4 = {X1 <= X2 <= X3 <= X4 < nb}.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define SMX_HD __host__ __device__ __forceinline__
#else
#include <cmath>
#define SMX_HD inline
#endif

namespace smx {

// MAP_CUBE is internal: one sub-orthotope of MAP_REC_LAUNCH, launched alone.
enum MapKind { MAP_LAMBDA = 0, MAP_BBOX = 1, MAP_LINEAR = 2, MAP_BELOW = 3, MAP_REC = 4, MAP_REC_LAUNCH = 5, MAP_CUBE = 6 };

// floor(log2 v), v >= 1.  The paper's bit-level form (Sec. III-A) counts from
// the word size W: floor(log2 v) = (W - 1) - clz(v), 2^floor(log2 v) = 1 << that.
SMX_HD int floor_log2_u32(uint32_t v) { return 31 - __builtin_clz(v); }

SMX_HD int ceil_log2_u64(uint64_t v) {
    int l = 0;
    while ((uint64_t(1) << l) < v) ++l;
    return l;
}

// Geometry shared by host sizing and device evaluation.
struct MapGeom {
    int32_t nb;     // tiles per dimension
    int32_t lg;     // log2 of nb' = next power of two >= nb (lambda and recursive
                    // maps); MAP_CUBE: log2 of the sub-orthotope's side
    uint32_t main;  // lambda3: blocks of the orthotope Pi3 (before the plane grid)
    uint32_t map;   // MapKind of the launch
    uint64_t G;     // logical blocks launched
    int32_t dim;    // m, the simplex dimension
    int32_t c0, c1, c2, c3;  // MAP_CUBE: corner-coordinate origin of the sub-orthotope
    uint64_t off;   // MAP_CUBE: position of its first block in the whole set
};

// ---------------------------------------------------------------- lambda2
// Sec. III-A.  Parallel space (nb'/2) x (nb'+1), linearised x fastest.  Rows
// 1..nb'-1: b = 2^floor(log2 w_y), q = floor(w_x / b),
// lambda(w) = (w_x + q b, w_y + 2 q b), a tile strictly above the diagonal.
// Rows 0 and nb' carry the diagonal: (w_x, w_x) and (nb'/2 + w_x, nb'/2 + w_x).
// nb' = 1 is a single block mapped to (0, 0).
SMX_HD uint64_t lambda2_blocks(int lg) {
    return lg == 0 ? 1 : (uint64_t(1) << (lg - 1)) * ((uint64_t(1) << lg) + 1);
}

SMX_HD bool lambda2(uint32_t id, int lg, int nb, int &X, int &Y) {
    if (lg == 0) {
        X = 0;
        Y = 0;
        return nb > 0;
    }
    const int h = lg - 1;
    const uint32_t wx = id & ((1u << h) - 1u);
    const uint32_t wy = id >> h;
    uint32_t x, y;
    if (wy == 0) {
        x = wx;
        y = wx;
    } else if (wy == (1u << lg)) {
        x = (1u << h) + wx;
        y = x;
    } else {
        const int L = floor_log2_u32(wy);
        const uint32_t q = wx >> L;
        x = wx + (q << L);
        y = wy + (q << (L + 1));
    }
    X = int(x);
    Y = int(y);
    return y < uint32_t(nb);  // x <= y
}

// The same parallel space Pi2 enumerated with w_y fastest ("column-major"):
// ids [0, (nb'/2) nb') are (w_x, w_y) = (id >> lg, id mod nb'), w_y = 0 the
// first diagonal row; the last nb'/2 ids are the row w_y = nb'.  lambda2 itself
// is unchanged.  Consecutive ids of one level (w_y in [b, 2b)) map to
// consecutive Y at a fixed X: a strip of tiles along one row panel.
SMX_HD uint32_t lambda2_cm_to_xfast(uint32_t id, int lg) {
    if (lg == 0) return id;
    const int h = lg - 1;
    const uint32_t body = 1u << (h + lg);
    const uint32_t wx = id < body ? id >> lg : id - body;
    const uint32_t wy = id < body ? id & ((1u << lg) - 1u) : 1u << lg;
    return (wy << h) | wx;
}

SMX_HD bool lambda2_cm(uint32_t id, int lg, int nb, int &X, int &Y) {
    return lambda2(lambda2_cm_to_xfast(id, lg), lg, nb, X, Y);
}

// Pi2 in patches of 2^pxl (w_x) x 2^pyl (w_y) ids (clamped to nb'/2 x nb'),
// w_y fastest inside a patch, the patches with their w_y index fastest; the
// row w_y = nb' comes last.  Inside one level a patch of Pi2 is a patch of
// tiles of one cross square (X = w_x + q b, Y = w_y + 2 q b), so consecutive
// ids reuse 2^pxl row panels and 2^pyl column panels.
SMX_HD uint32_t lambda2_patch_to_xfast(uint32_t id, int lg, int pxl, int pyl) {
    if (lg == 0) return id;
    const int h = lg - 1;
    const uint32_t body = 1u << (h + lg);
    if (id >= body) return (1u << (h + lg)) | (id - body);
    const int px = pxl < h ? pxl : h, py = pyl < lg ? pyl : lg;
    const uint32_t p = id >> (px + py), r = id & ((1u << (px + py)) - 1u);
    const uint32_t pwy = p & ((1u << (lg - py)) - 1u), pwx = p >> (lg - py);
    const uint32_t wy = (pwy << py) | (r & ((1u << py) - 1u)), wx = (pwx << px) | (r >> py);
    return (wy << h) | wx;
}

// ---------------------------------------------------------------- lambda3
// Sec. III-C, two recursion branches.  Pi3 = (nb'/2) x (nb'/2) x (nb'/2 + nb'/4),
// linearised x fastest.  Target of Pi3: {X <= Y < Z}.  The first nb'/2
// z-slices are the main cube, level b = nb'/2, offset o = 0, (u, v, w) = w.
// The other slices are a slab reusing lambda2's level of w_y:
// w = w_z - nb'/2, b = 2^floor(log2 w_y), q = floor(w_x / b), u = w_x - q b,
// v = w_y - b, o = 2 q b; blocks with w_y = 0 or w >= b are filtered.  Each b^3
// block-cube folds across its diagonal plane onto the cross cube
// {o <= X < o+b <= Z < o+2b} of the tetrahedron:
//   v <  w : (o + u, o + b + v, o + b + w)
//   v >= w : (o + w, o + v,     o + b + u)
// Blocks past Pi3 form a lambda2 grid over nb whose tile (X, Y) becomes the
// plane tile (X, Y, Y).
SMX_HD uint32_t lambda3_main_blocks(int lg) {
    if (lg == 0) return 0;
    const uint32_t half = 1u << (lg - 1);
    return half * half * (half + (half >> 1));
}

SMX_HD bool lambda3(uint32_t id, int lg, int nb, uint32_t main, int &X, int &Y, int &Z) {
    if (id < main) {
        const int h = lg - 1;
        const uint32_t half = 1u << h;
        const uint32_t wx = id & (half - 1u);
        const uint32_t wy = (id >> h) & (half - 1u);
        const uint32_t wz = id >> (2 * h);
        uint32_t u, v, w, b, o;
        if (wz < half) {
            u = wx;
            v = wy;
            w = wz;
            b = half;
            o = 0;
        } else {
            w = wz - half;
            if (wy == 0) return false;
            const int L = floor_log2_u32(wy);
            b = 1u << L;
            if (w >= b) return false;
            const uint32_t q = wx >> L;
            u = wx - (q << L);
            v = wy - b;
            o = q << (L + 1);
        }
        uint32_t x, y, z;
        if (v < w) {
            x = o + u;
            y = o + b + v;
            z = o + b + w;
        } else {
            x = o + w;
            y = o + v;
            z = o + b + u;
        }
        X = int(x);
        Y = int(y);
        Z = int(z);
        return z < uint32_t(nb);
    }
    int x2, y2;
    if (!lambda2(id - main, lg, nb, x2, y2)) return false;
    X = x2;
    Y = y2;
    Z = y2;
    return true;
}

// ---------------------------------------------------------------- linear
// Linear enumeration (Sec. I): block k is the k-th tile of T2 listed by Y
// then X, or of T3 listed by Z, Y, X.  The root of the quadratic (cubic) is
// taken in FP32 and then corrected with exact integer comparisons, so the
// result is exact for every k although FP32 roots are not once k > 2^24.
SMX_HD uint64_t tri_u64(uint64_t y) { return y * (y + 1) / 2; }
SMX_HD uint64_t tet_u64(uint64_t z) { return z * (z + 1) * (z + 2) / 6; }

SMX_HD uint32_t tri_root(uint64_t k) {
#if defined(__HIP_DEVICE_COMPILE__)
    const float f = __builtin_sqrtf(8.0f * float(k) + 1.0f);
#else
    const float f = std::sqrt(8.0f * float(k) + 1.0f);
#endif
    float g = (f - 1.0f) * 0.5f;
    uint64_t y = g > 0.0f ? uint64_t(g) : 0;
    while (y > 0 && tri_u64(y) > k) --y;
    while (tri_u64(y + 1) <= k) ++y;
    return uint32_t(y);
}

SMX_HD uint32_t tet_root(uint64_t k) {
#if defined(__HIP_DEVICE_COMPILE__)
    const float f = cbrtf(6.0f * float(k));
#else
    const float f = std::cbrt(6.0f * float(k));
#endif
    uint64_t z = f > 1.0f ? uint64_t(f) - 1 : 0;
    while (z > 0 && tet_u64(z) > k) --z;
    while (tet_u64(z + 1) <= k) ++z;
    return uint32_t(z);
}

SMX_HD void linear2(uint32_t k, int &X, int &Y) {
    const uint32_t y = tri_root(k);
    Y = int(y);
    X = int(uint64_t(k) - tri_u64(y));
}

SMX_HD void linear3(uint32_t k, int &X, int &Y, int &Z) {
    const uint32_t z = tet_root(k);
    const uint64_t r = uint64_t(k) - tet_u64(z);
    const uint32_t y = tri_root(r);
    Z = int(z);
    Y = int(y);
    X = int(r - tri_u64(y));
}

// 4-simplex: block k is the k-th tile of T4 listed by X4, X3, X2, X1.
SMX_HD uint64_t pen_u64(uint64_t w) { return w * (w + 1) * (w + 2) * (w + 3) / 24; }

SMX_HD uint32_t pen_root(uint64_t k) {
#if defined(__HIP_DEVICE_COMPILE__)
    const float f = __builtin_sqrtf(__builtin_sqrtf(24.0f * float(k)));
#else
    const float f = std::sqrt(std::sqrt(24.0f * float(k)));
#endif
    uint64_t w = f > 2.0f ? uint64_t(f) - 2 : 0;
    while (w > 0 && pen_u64(w) > k) --w;
    while (pen_u64(w + 1) <= k) ++w;
    return uint32_t(w);
}

SMX_HD void linear4(uint32_t k, int X[4]) {
    const uint32_t w = pen_root(k);
    int t[3];
    linear3(uint32_t(uint64_t(k) - pen_u64(w)), t[0], t[1], t[2]);
    X[0] = t[0];
    X[1] = t[1];
    X[2] = t[2];
    X[3] = int(w);
}

// ---------------------------------------------------------------- from below
// "Approach n from below" (Sec. III-A): nb is split into its binary digits,
// largest first, segments [o, o + m) with m = 2^floor(log2 rest).  All sizes
// below are powers of two, so the lambda maps inside them filter nothing in 2-D.
//   2-simplex, per segment: lambda2 of m on its diagonal triangle, then the
//     rectangle [o, o + m) x [o + m, nb) under the identity (x fastest).
//   3-simplex, per segment: lambda3 of m (its tetrahedron), then the prism
//     {x <= y in the segment, z above} = lambda2(m) x identity, then the prism
//     {x in the segment, y <= z above} = identity x (2-simplex from below of
//     the rest).
// Decoding walks the segments (at most popcount(nb) steps, block uniform).
SMX_HD uint64_t below2_blocks(uint64_t nb) { return nb * (nb + 1) / 2; }

SMX_HD bool below2(uint64_t id, uint32_t nb, int &X, int &Y) {
    uint32_t o = 0, rem = nb;
    while (rem != 0) {
        const int L = floor_log2_u32(rem);
        const uint32_t m = 1u << L, r = rem - m;
        const uint64_t tri = uint64_t(m) * (m + 1) / 2;
        if (id < tri) {
            int x, y;
            lambda2(uint32_t(id), L, int(m), x, y);
            X = int(o) + x;
            Y = int(o) + y;
            return true;
        }
        id -= tri;
        const uint64_t rect = uint64_t(m) * r;
        if (id < rect) {
            X = int(o + uint32_t(id & (m - 1)));
            Y = int(o + m + uint32_t(id >> L));
            return true;
        }
        id -= rect;
        o += m;
        rem = r;
    }
    return false;
}

SMX_HD uint64_t below3_blocks(uint64_t nb) {
    uint64_t tot = 0, rem = nb;
    while (rem != 0) {
        int L = 0;
        while ((uint64_t(2) << L) <= rem) ++L;
        const uint64_t m = uint64_t(1) << L, r = rem - m;
        tot += lambda3_main_blocks(L) + lambda2_blocks(L) + lambda2_blocks(L) * r + m * (r * (r + 1) / 2);
        rem = r;
    }
    return tot;
}

SMX_HD bool below3(uint64_t id, uint32_t nb, int &X, int &Y, int &Z) {
    uint32_t o = 0, rem = nb;
    while (rem != 0) {
        const int L = floor_log2_u32(rem);
        const uint32_t m = 1u << L, r = rem - m;
        const uint32_t main = lambda3_main_blocks(L);
        const uint64_t p2 = lambda2_blocks(L);
        const uint64_t tet = uint64_t(main) + p2;
        if (id < tet) {
            int x, y, z;
            if (!lambda3(uint32_t(id), L, int(m), main, x, y, z)) return false;
            X = int(o) + x;
            Y = int(o) + y;
            Z = int(o) + z;
            return true;
        }
        id -= tet;
        const uint64_t pa = p2 * r;
        if (id < pa) {
            const uint64_t z = id / p2;
            int x, y;
            lambda2(uint32_t(id - z * p2), L, int(m), x, y);
            X = int(o) + x;
            Y = int(o) + y;
            Z = int(o + m + uint32_t(z));
            return true;
        }
        id -= pa;
        const uint64_t pb = uint64_t(m) * (uint64_t(r) * (r + 1) / 2);
        if (id < pb) {
            int y, z;
            below2(id >> L, r, y, z);
            X = int(o + uint32_t(id & (m - 1)));
            Y = int(o + m) + y;
            Z = int(o + m) + z;
            return true;
        }
        id -= pb;
        o += m;
        rem = r;
    }
    return false;
}

// ---------------------------------------------------------------- recursive
// The recursive orthotope sets of Sec. III-B, mapped level by level in
// O(log n) steps (the map the paper describes before setting it aside for its
// cost in recursive calls).  They live in the paper's corner coordinates p
// (p_1 + ... + p_m <= nb' - 1, the orthogonal corner at 0): the map of a simplex
// of side s at relative origin c is the cube phi(w, c) of side s/2 at c,
// followed by m maps of side s/2 at c + (s/2) e_d, one per axis (for m = 3 the
// sides and the top of the cube), down to single blocks.  Blocks are numbered
// depth first in that order: V(1) = 1, V(s) = (s/2)^m + m V(s/2), so that
// V(nb') = nb'(nb'+1)/2 for m = 2 (every block inside) and (nb'^3 + 4 3^lg) / 5
// for m = 3 (extra volume -> 1/5).  A corner point p is the tile
// (p_1, p_1 + p_2[, p_1 + p_2 + p_3]) of T2 / T3 -- a unimodular shear, so a
// cover of the corner simplex is a cover of the tile set; blocks whose last
// coordinate reaches nb (outside the simplex, or past nb when nb' > nb) are
// filtered.  Decoding walks down from the top: at side s the block is in the
// cube if id < (s/2)^m, else in branch floor((id - (s/2)^m) / V(s/2)), found by
// comparisons; V(s/2) = (V(s) - (s/2)^m) / m.
SMX_HD uint64_t rec_blocks(int m, int lg) {
    uint64_t v = 1;
    for (int l = 1; l <= lg; ++l) v = (uint64_t(1) << (m * (l - 1))) + uint64_t(m) * v;
    return v;
}

SMX_HD bool rec2(uint32_t id, int lg, int nb, uint32_t V, int &X, int &Y) {
    uint32_t a = 0, b = 0;
    for (int l = lg; l > 0; --l) {
        const int h = l - 1;
        const uint32_t cube = 1u << (2 * h);
        if (id < cube) {
            a += id & ((1u << h) - 1u);
            b += id >> h;
            break;
        }
        id -= cube;
        const uint32_t vh = (V - cube) >> 1;
        if (id < vh) {
            a += 1u << h;
        } else {
            b += 1u << h;
            id -= vh;
        }
        V = vh;
    }
    X = int(a);
    Y = int(a + b);
    return a + b < uint32_t(nb);
}

SMX_HD bool rec3(uint32_t id, int lg, int nb, uint32_t V, int &X, int &Y, int &Z) {
    uint32_t a = 0, b = 0, c = 0;
    for (int l = lg; l > 0; --l) {
        const int h = l - 1;
        const uint32_t cube = 1u << (3 * h);
        if (id < cube) {
            const uint32_t mask = (1u << h) - 1u;
            a += id & mask;
            b += (id >> h) & mask;
            c += id >> (2 * h);
            break;
        }
        id -= cube;
        const uint32_t vh = (V - cube) / 3u;
        if (id < vh) {
            a += 1u << h;
        } else if (id < 2 * vh) {
            b += 1u << h;
            id -= vh;
        } else {
            c += 1u << h;
            id -= 2 * vh;
        }
        V = vh;
    }
    X = int(a);
    Y = int(a + b);
    Z = int(a + b + c);
    return a + b + c < uint32_t(nb);
}

SMX_HD bool rec4(uint32_t id, int lg, int nb, uint32_t V, int X[4]) {
    uint32_t p0 = 0, p1 = 0, p2 = 0, p3 = 0;
    for (int l = lg; l > 0; --l) {
        const int h = l - 1;
        const uint32_t cube = 1u << (4 * h);
        if (id < cube) {
            const uint32_t mask = (1u << h) - 1u;
            p0 += id & mask;
            p1 += (id >> h) & mask;
            p2 += (id >> (2 * h)) & mask;
            p3 += id >> (3 * h);
            break;
        }
        id -= cube;
        const uint32_t vh = (V - cube) >> 2;
        if (id < vh) {
            p0 += 1u << h;
        } else if (id < 2 * vh) {
            p1 += 1u << h;
            id -= vh;
        } else if (id < 3 * vh) {
            p2 += 1u << h;
            id -= 2 * vh;
        } else {
            p3 += 1u << h;
            id -= 3 * vh;
        }
        V = vh;
    }
    X[0] = int(p0);
    X[1] = int(p0 + p1);
    X[2] = int(p0 + p1 + p2);
    X[3] = int(p0 + p1 + p2 + p3);
    return p0 + p1 + p2 + p3 < uint32_t(nb);
}

// One sub-orthotope of the recursive set on its own launch (MAP_CUBE): block
// id of the cube of side 2^g.lg at corner origin (c0, c1[, c2]), x fastest.
SMX_HD bool cube2(uint32_t id, const MapGeom &g, int &X, int &Y) {
    const uint32_t a = uint32_t(g.c0) + (id & ((1u << g.lg) - 1u));
    const uint32_t b = uint32_t(g.c1) + (id >> g.lg);
    X = int(a);
    Y = int(a + b);
    return a + b < uint32_t(g.nb);
}

SMX_HD bool cube3(uint32_t id, const MapGeom &g, int &X, int &Y, int &Z) {
    const uint32_t mask = (1u << g.lg) - 1u;
    const uint32_t a = uint32_t(g.c0) + (id & mask);
    const uint32_t b = uint32_t(g.c1) + ((id >> g.lg) & mask);
    const uint32_t c = uint32_t(g.c2) + (id >> (2 * g.lg));
    X = int(a);
    Y = int(a + b);
    Z = int(a + b + c);
    return a + b + c < uint32_t(g.nb);
}

SMX_HD bool cube4(uint32_t id, const MapGeom &g, int X[4]) {
    const uint32_t mask = (1u << g.lg) - 1u;
    const uint32_t a = uint32_t(g.c0) + (id & mask);
    const uint32_t b = uint32_t(g.c1) + ((id >> g.lg) & mask);
    const uint32_t c = uint32_t(g.c2) + ((id >> (2 * g.lg)) & mask);
    const uint32_t d = uint32_t(g.c3) + (id >> (3 * g.lg));
    X[0] = int(a);
    X[1] = int(a + b);
    X[2] = int(a + b + c);
    X[3] = int(a + b + c + d);
    return a + b + c + d < uint32_t(g.nb);
}

// ---------------------------------------------------------------- lambda4
// The 4-simplex map built on the r = 1/2, beta = 2 recursive set of Sec. III-D
// (the paper gives that set and its volume (n^4 - n)/14, not a map).  T4 is
// split into T4s = {X1 <= X2 <= X3 < X4} and the plane X3 = X4 (a copy of T3).
// A tuple of T4s belongs to the node of the binary recursion on [0, nb') --
// offset o, size 2b -- where X1 and X4 first fall on different halves
// L = [o, o+b), H = [o+b, o+2b); its cross region is
//   R3 = {X1 <= X2 <= X3 in L, X4 in H}     b C(b+2, 3) tiles
//   R2 = {X1 <= X2 in L, X3 < X4 in H}      C(b+1, 2) C(b, 2)
//   R1 = {X1 in L, X2 <= X3 < X4 in H}      b C(b+1, 3)
// b^2 (b+1)(7b-1)/12 <= b^4 tiles.  Each node owns one b^4 orthotope of blocks:
// level l (b = nb'/2^(l+1)) holds 2^l nodes, 2^(4 lg - 3l - 4) blocks, and the
// levels add up to (nb'^4 - nb')/14.  Within a node the leading blocks unrank
// R3, R2, R1 in turn (the sorted triples and pairs by FP32 roots with exact
// 32-bit corrections, the free coordinate fastest); the rest are filtered (the 5/7
// extra volume of the set).  Blocks past the orthotopes form a lambda3 grid over
// nb whose tile (X, Y, Z) becomes (X, Y, Z, Z).  The level is found in at most
// lg block-uniform steps.
// Unranking inside a lambda4 node (ranks below 2^27, values below 2^8): an
// FP32 estimate, then exact 32-bit corrections.  tri32: largest y with
// y(y+1)/2 <= k; tet32: largest z with z(z+1)(z+2)/6 <= k; quo32: floor(k / q).
SMX_HD uint32_t tri32(uint32_t k) {
#if defined(__HIP_DEVICE_COMPILE__)
    const float f = __builtin_sqrtf(8.0f * float(k) + 1.0f);
#else
    const float f = std::sqrt(8.0f * float(k) + 1.0f);
#endif
    uint32_t y = uint32_t((f - 1.0f) * 0.5f);
    while (y > 0 && y * (y + 1) / 2 > k) --y;
    while ((y + 1) * (y + 2) / 2 <= k) ++y;
    return y;
}

SMX_HD uint32_t tet32(uint32_t k) {
#if defined(__HIP_DEVICE_COMPILE__)
    // 6k to the power 1/3 by the hardware base-2 logarithm and exponential
    const float f = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(6.0f * float(k) + 1.0f) * (1.0f / 3.0f));
#else
    const float f = std::cbrt(6.0f * float(k) + 1.0f);
#endif
    uint32_t z = f > 1.0f ? uint32_t(f) - 1 : 0;
    while (z > 0 && z * (z + 1) * (z + 2) / 6 > k) --z;
    while ((z + 1) * (z + 2) * (z + 3) / 6 <= k) ++z;
    return z;
}

SMX_HD uint32_t quo32(uint32_t k, uint32_t q) {
    uint32_t p = uint32_t(float(k) / float(q));
    while (p > 0 && p * q > k) --p;
    while ((p + 1) * q <= k) ++p;
    return p;
}

// Sorted triple x <= y <= z of rank t (listed by z, then y, then x).
SMX_HD void unrank3(uint32_t t, uint32_t &x, uint32_t &y, uint32_t &z) {
    z = tet32(t);
    const uint32_t r = t - z * (z + 1) * (z + 2) / 6;
    y = tri32(r);
    x = r - y * (y + 1) / 2;
}

SMX_HD uint64_t lambda4_main_blocks(int lg) {
    uint64_t v = 0;
    for (int l = 0; l < lg; ++l) v += uint64_t(1) << (4 * lg - 3 * l - 4);
    return v;
}

SMX_HD bool lambda4(uint32_t id, int lg, int nb, uint32_t main, int X[4]) {
    if (id >= main) {
        int x, y, z;
        if (!lambda3(id - main, lg, nb, lambda3_main_blocks(lg), x, y, z)) return false;
        X[0] = x;
        X[1] = y;
        X[2] = z;
        X[3] = z;
        return true;
    }
    int l = 0;
    uint32_t r = id;
    for (;;) {
        const uint32_t sz = 1u << (4 * lg - 3 * l - 4);
        if (r < sz) break;
        r -= sz;
        ++l;
    }
    const int h = lg - l - 1;
    const uint32_t b = 1u << h;
    const uint32_t o = (r >> (4 * h)) << (h + 1);
    uint32_t loc = r & ((1u << (4 * h)) - 1u);
    uint32_t x, y, z;
    const uint32_t n3 = b * (b * (b + 1) * (b + 2) / 6);
    if (loc < n3) {
        unrank3(loc >> h, x, y, z);
        X[0] = int(o + x);
        X[1] = int(o + y);
        X[2] = int(o + z);
        X[3] = int(o + b + (loc & (b - 1u)));
        return X[3] < nb;
    }
    loc -= n3;
    const uint32_t P = b * (b + 1) / 2, Q = b * (b - 1) / 2;
    if (loc < P * Q) {
        const uint32_t p = quo32(loc, Q), s = loc - p * Q;
        const uint32_t c = tri32(p), e1 = tri32(s);  // (a <= c) of rank p; strict (d < e) of rank s: e = e1 + 1
        X[0] = int(o + (p - c * (c + 1) / 2));
        X[1] = int(o + c);
        X[2] = int(o + b + (s - e1 * (e1 + 1) / 2));
        X[3] = int(o + b + e1 + 1);
        return X[3] < nb;
    }
    loc -= P * Q;
    const uint32_t n1 = b * ((b + 1) * b * (b - 1) / 6);
    if (loc < n1) {
        unrank3(loc >> h, x, y, z);  // X2 <= X3 <= X4 - 1 in H
        X[0] = int(o + (loc & (b - 1u)));
        X[1] = int(o + b + x);
        X[2] = int(o + b + y);
        X[3] = int(o + b + z + 1);
        return X[3] < nb;
    }
    return false;
}

// ---------------------------------------------------------------- XCD order
// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each with
// its own L2.  Renumbering dispatch index b so that XCD (b mod 8) receives one
// contiguous range of logical blocks keeps neighbouring tiles, which share
// input rows, in one L2.  A bijection on [0, G).
SMX_HD uint32_t xcd_remap(uint32_t b, uint32_t G) {
    const uint32_t chunk = G >> 3, rem = G & 7u, x = b & 7u, s = b >> 3;
    return x * chunk + (x < rem ? x : rem) + s;
}

}  // namespace smx
