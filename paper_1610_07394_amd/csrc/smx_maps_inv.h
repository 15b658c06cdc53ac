// Inverses of the block-space maps: the launched block that a map sends to a
// given tile (the tile must lie in the target simplex).  They follow the
// recursive sets rather than undoing the forward formulas step by step: a pair
// X < Y belongs to the level b = 2^L of the 2-simplex recursion where
// L = msb(X xor Y) (the highest bit where the indices part), and to its square
// q = X >> (L+1); a triple X <= Y < Z belongs to the level of msb(X xor Z) of the
// 3-simplex recursion, on the first prism when Y reaches the upper half.
#pragma once
#include "smx_maps.h"

namespace smx {

SMX_HD int msb_u32(uint32_t v) { return 31 - __builtin_clz(v); }

// lambda2 (Sec. III-A): block index of tile (X, Y), X <= Y < nb, grid of nb' = 2^lg.
SMX_HD uint64_t lambda2_inv(int lg, uint32_t X, uint32_t Y) {
    if (lg == 0) return 0;
    const uint32_t half = 1u << (lg - 1);
    if (X == Y) return X < half ? X : (uint64_t(1u << lg) * half + (X - half));
    const int L = msb_u32(X ^ Y);
    const uint32_t b = 1u << L, q = X >> (L + 1);
    const uint32_t wx = X - q * b, wy = Y - 2 * q * b;
    return uint64_t(wy) * half + wx;
}

// lambda3 (Sec. III-C reading): tile (X, Y, Z), X <= Y <= Z < nb.  Tiles of the
// plane Y = Z come from the lambda2 grid appended after the main orthotope.
SMX_HD uint64_t lambda3_inv(int lg, uint32_t main, uint32_t X, uint32_t Y, uint32_t Z) {
    if (Y == Z) return uint64_t(main) + lambda2_inv(lg, X, Y);
    const uint32_t half = 1u << (lg - 1);
    const int L = msb_u32(X ^ Z);
    const uint32_t b = 1u << L, o = (X >> (L + 1)) << (L + 1);
    uint32_t u, v, w;
    if (Y >= o + b) {  // first prism: v < w
        u = X - o;
        v = Y - o - b;
        w = Z - o - b;
    } else {           // second prism: v >= w
        w = X - o;
        v = Y - o;
        u = Z - o - b;
    }
    uint32_t wx = u, wy = v, wz = w;
    if (b != half) {   // slab: level b, square q of lambda2's row band
        wx = u + (o / (2 * b)) * b;
        wy = v + b;
        wz = w + half;
    }
    return uint64_t(wx) + uint64_t(half) * (uint64_t(wy) + uint64_t(half) * wz);
}

// Linear enumeration (Sec. I): the rank of the tile in the listing by the last
// coordinate, then the previous ones.
SMX_HD uint64_t linear2_inv(uint32_t X, uint32_t Y) { return uint64_t(Y) * (Y + 1) / 2 + X; }
SMX_HD uint64_t linear3_inv(uint32_t X, uint32_t Y, uint32_t Z) {
    return uint64_t(Z) * (Z + 1) * (Z + 2) / 6 + uint64_t(Y) * (Y + 1) / 2 + X;
}

}  // namespace smx
