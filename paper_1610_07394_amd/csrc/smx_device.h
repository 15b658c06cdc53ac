// Device-side helpers shared by the kernels: launch geometry, element ids,
// SplitMix64, wave64 reductions and the statistics / energy slots.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smx_maps.h"

namespace smx {

constexpr int kWave = 64;

// Checked builds (compiled with SMX_CHECKED=1 into a separate library): device
// checks that record a violation in a flag word of the translation unit and
// skip the access instead of performing it.  Bit kCheckMap: a map produced a
// tile outside the simplex; bit kCheckStore: a kernel was about to store an
// element outside the simplex (an unmasked store on a tile it took for
// interior).  In normal builds the checks compile to nothing.
#ifndef SMX_CHECKED
#define SMX_CHECKED 0
#endif
constexpr unsigned kCheckMap = 1u, kCheckStore = 2u;
#if SMX_CHECKED
static __device__ unsigned int g_check_flags;
#endif
__device__ __forceinline__ bool smx_check(bool ok, unsigned bit) {
#if SMX_CHECKED
    if (!ok) atomicOr(&g_check_flags, bit);
    return ok;
#else
    (void)ok;
    (void)bit;
    return true;
#endif
}
// Statistics and energy partials are accumulated with atomics spread over
// kSlots addresses, one 128-byte line apart, so that millions of blocks do not
// serialise on one address.  A finalize kernel sums the slots.
constexpr int kSlots = 256;
constexpr int kSlotStride = 16;  // 16 x 8 bytes = one 128-byte line
constexpr size_t kSlotBytes = size_t(kSlots) * kSlotStride * 8;

// Logical index of this block on a 1-D or 2-D launch of G blocks (2-D when
// G * threads would overflow the 32-bit per-dimension thread count).
__device__ __forceinline__ uint64_t launch_index() {
    return uint64_t(blockIdx.y) * gridDim.x + blockIdx.x;
}

// True for the tail blocks of a 2-D launch (logical index >= G), which hold no
// position in a tile dump.
template <int MAP>
__device__ __forceinline__ bool launch_tail(const MapGeom &g) {
    return MAP != MAP_BBOX && launch_index() >= g.G;
}

// tile2_decode / tile3_decode: the tile of a given logical block id (< G), for
// kernels that decode ids themselves; the bounding box's id is the row-major
// rank of its grid position (X fastest).
template <int MAP>
__device__ __forceinline__ bool tile2_decode(const MapGeom &g, uint32_t id, uint64_t &lin, int &X, int &Y) {
    lin = id;
    if (MAP == MAP_BBOX) {
        const uint32_t nb = uint32_t(g.nb), q = id / nb;
        X = int(id - q * nb);
        Y = int(q);
        return X <= Y;
    }
    if (MAP == MAP_LAMBDA) return lambda2(id, g.lg, g.nb, X, Y);
    if (MAP == MAP_BELOW) return below2(id, uint32_t(g.nb), X, Y);
    if (MAP == MAP_REC) return rec2(id, g.lg, g.nb, uint32_t(g.G), X, Y);
    if (MAP == MAP_CUBE) {
        lin = g.off + id;
        return cube2(id, g, X, Y);
    }
    linear2(id, X, Y);
    return true;
}

template <int MAP>
__device__ __forceinline__ bool tile3_decode(const MapGeom &g, uint32_t id, uint64_t &lin, int &X, int &Y,
                                             int &Z) {
    lin = id;
    if (MAP == MAP_BBOX) {
        const uint32_t nb = uint32_t(g.nb), q = id / nb, q2 = q / nb;
        X = int(id - q * nb);
        Y = int(q - q2 * nb);
        Z = int(q2);
        return X <= Y && Y <= Z;
    }
    if (MAP == MAP_LAMBDA) return lambda3(id, g.lg, g.nb, g.main, X, Y, Z);
    if (MAP == MAP_BELOW) return below3(id, uint32_t(g.nb), X, Y, Z);
    if (MAP == MAP_REC) return rec3(id, g.lg, g.nb, uint32_t(g.G), X, Y, Z);
    if (MAP == MAP_CUBE) {
        lin = g.off + id;
        return cube3(id, g, X, Y, Z);
    }
    linear3(id, X, Y, Z);
    return true;
}

// Tile of this block under map MAP.  Returns false for a filtered block (and
// for the tail of a 2-D launch, where lin >= G).  `lin` receives the logical
// block index (the dump position).  XCD: renumber the dispatch order so that
// each XCD takes one contiguous range of logical blocks.  The bounding box is
// the hardware 2-D / 3-D grid itself (identity map, no renumbering).
template <int MAP, bool XCD>
__device__ __forceinline__ bool tile2_raw(const MapGeom &g, uint64_t &lin, int &X, int &Y) {
    if (MAP == MAP_BBOX) {
        X = int(blockIdx.x);
        Y = int(blockIdx.y);
        lin = uint64_t(Y) * uint64_t(g.nb) + uint64_t(X);
        return X <= Y;
    }
    lin = uint64_t(blockIdx.y) * gridDim.x + blockIdx.x;
    if (lin >= g.G) return false;
    const uint32_t id = XCD ? xcd_remap(uint32_t(lin), uint32_t(g.G)) : uint32_t(lin);
    return tile2_decode<MAP>(g, id, lin, X, Y);
}

template <int MAP, bool XCD>
__device__ __forceinline__ bool tile3_raw(const MapGeom &g, uint64_t &lin, int &X, int &Y, int &Z) {
    if (MAP == MAP_BBOX) {
        X = int(blockIdx.x);
        Y = int(blockIdx.y);
        Z = int(blockIdx.z);
        lin = (uint64_t(Z) * uint64_t(g.nb) + uint64_t(Y)) * uint64_t(g.nb) + uint64_t(X);
        return X <= Y && Y <= Z;
    }
    lin = uint64_t(blockIdx.y) * gridDim.x + blockIdx.x;
    if (lin >= g.G) return false;
    const uint32_t id = XCD ? xcd_remap(uint32_t(lin), uint32_t(g.G)) : uint32_t(lin);
    return tile3_decode<MAP>(g, id, lin, X, Y, Z);
}

// 4-simplex tiles (X[0] <= X[1] <= X[2] <= X[3]).  There is no 4-D hardware
// grid: every map, the bounding box included, runs on a 1-D (or 2-D) launch,
// and the bounding box decodes its block index with divisions by nb.  The
// from-below map is not defined for m = 4 (the host rejects it).
//
// tile4_decode: the tile of logical block id (< G); lin gets the id (offset by
// the cube's first id for one launch of the launch-per-cube recursion).
template <int MAP>
__device__ __forceinline__ bool tile4_decode(const MapGeom &g, uint32_t id, uint64_t &lin, int X[4]) {
    lin = id;
    if (MAP == MAP_BBOX) {
        const uint32_t nb = uint32_t(g.nb);
        uint32_t r = id;
        for (int d = 0; d < 4; ++d) {
            const uint32_t q = r / nb;
            X[d] = int(r - q * nb);
            r = q;
        }
        return X[0] <= X[1] && X[1] <= X[2] && X[2] <= X[3];
    }
    if (MAP == MAP_LAMBDA) return lambda4(id, g.lg, g.nb, g.main, X);
    if (MAP == MAP_REC) return rec4(id, g.lg, g.nb, uint32_t(g.G), X);
    if (MAP == MAP_CUBE) {
        lin = g.off + id;
        return cube4(id, g, X);
    }
    if (MAP == MAP_LINEAR) {
        linear4(id, X);
        return true;
    }
    return false;
}

template <int MAP, bool XCD>
__device__ __forceinline__ bool tile4_raw(const MapGeom &g, uint64_t &lin, int X[4]) {
    lin = uint64_t(blockIdx.y) * gridDim.x + blockIdx.x;
    if (lin >= g.G) return false;
    const uint32_t id = XCD ? xcd_remap(uint32_t(lin), uint32_t(g.G)) : uint32_t(lin);
    return tile4_decode<MAP>(g, id, lin, X);
}

// The map entry points used by the kernels: the raw map, then (checked builds)
// the tile's place in the simplex.
template <int MAP, bool XCD>
__device__ __forceinline__ bool tile2_of(const MapGeom &g, uint64_t &lin, int &X, int &Y) {
    bool ok = tile2_raw<MAP, XCD>(g, lin, X, Y);
    if (SMX_CHECKED && ok) ok = smx_check(0 <= X && X <= Y && Y < g.nb, kCheckMap);
    return ok;
}

template <int MAP, bool XCD>
__device__ __forceinline__ bool tile3_of(const MapGeom &g, uint64_t &lin, int &X, int &Y, int &Z) {
    bool ok = tile3_raw<MAP, XCD>(g, lin, X, Y, Z);
    if (SMX_CHECKED && ok) ok = smx_check(0 <= X && X <= Y && Y <= Z && Z < g.nb, kCheckMap);
    return ok;
}

template <int MAP, bool XCD>
__device__ __forceinline__ bool tile4_of(const MapGeom &g, uint64_t &lin, int X[4]) {
    bool ok = tile4_raw<MAP, XCD>(g, lin, X);
    if (SMX_CHECKED && ok)
        ok = smx_check(0 <= X[0] && X[0] <= X[1] && X[1] <= X[2] && X[2] <= X[3] && X[3] < g.nb, kCheckMap);
    return ok;
}

// The tile of a given logical block id (< G), for kernels whose blocks take
// several tiles.
template <int MAP>
__device__ __forceinline__ bool tile2_of_id(const MapGeom &g, uint32_t id, uint64_t &lin, int &X, int &Y) {
    bool ok = tile2_decode<MAP>(g, id, lin, X, Y);
    if (SMX_CHECKED && ok) ok = smx_check(0 <= X && X <= Y && Y < g.nb, kCheckMap);
    return ok;
}

template <int MAP>
__device__ __forceinline__ bool tile3_of_id(const MapGeom &g, uint32_t id, uint64_t &lin, int &X, int &Y, int &Z) {
    bool ok = tile3_decode<MAP>(g, id, lin, X, Y, Z);
    if (SMX_CHECKED && ok) ok = smx_check(0 <= X && X <= Y && Y <= Z && Z < g.nb, kCheckMap);
    return ok;
}

template <int MAP>
__device__ __forceinline__ bool tile4_of_id(const MapGeom &g, uint32_t id, uint64_t &lin, int X[4]) {
    bool ok = tile4_decode<MAP>(g, id, lin, X);
    if (SMX_CHECKED && ok)
        ok = smx_check(0 <= X[0] && X[0] <= X[1] && X[1] <= X[2] && X[2] <= X[3] && X[3] < g.nb, kCheckMap);
    return ok;
}

// SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014): the output function
// applied to state x + golden-ratio increment.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Element ids (bijections onto [0, V)).
__device__ __forceinline__ uint64_t id_pair_le(uint64_t i, uint64_t j, uint64_t n) {
    return i * n - (i * (i - 1)) / 2 + (j - i);  // i = 0: (0 * -1) / 2 wraps to 0 correctly
}
__device__ __forceinline__ uint64_t id_pair_lt(uint64_t i, uint64_t j) { return (j * (j - 1)) / 2 + i; }
__device__ __forceinline__ uint64_t id_trip_le(uint64_t i, uint64_t j, uint64_t k) {
    return (k * (k + 1) * (k + 2)) / 6 + (j * (j + 1)) / 2 + i;
}
__device__ __forceinline__ uint64_t id_trip_lt(uint64_t i, uint64_t j, uint64_t k) {
    return (k * (k - 1) * (k - 2)) / 6 + (j * (j - 1)) / 2 + i;
}
__device__ __forceinline__ uint64_t id_quad_le(uint64_t i, uint64_t j, uint64_t k, uint64_t l) {
    return (l * (l + 1) * (l + 2) * (l + 3)) / 24 + (k * (k + 1) * (k + 2)) / 6 + (j * (j + 1)) / 2 + i;
}
__device__ __forceinline__ uint64_t id_quad_lt(uint64_t i, uint64_t j, uint64_t k, uint64_t l) {
    return (l * (l - 1) * (l - 2) * (l - 3)) / 24 + (k * (k - 1) * (k - 2)) / 6 + (j * (j - 1)) / 2 + i;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Block-wide sum of a per-thread value; the result is valid in thread 0.
template <typename T, int NTHREADS>
__device__ __forceinline__ T block_sum(T v, T *scratch /* NTHREADS / 64 entries */) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    T r = T(0);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < NTHREADS / kWave; ++w) r += scratch[w];
    }
    return r;
}

// Count and checksum the pairs i <= j (ids p(i, j), the packed index) of the
// tile rows [i0, i0 + rows) x columns [j0, j0 + cols), all threads of the block
// taking part.  Used by the statistics variants of the EDM kernels, after the
// tile is stored, so that the counting does not share registers with the tile
// arithmetic.
template <int NTHREADS>
__device__ __forceinline__ void tile_pairs_le_stats(int64_t i0, int64_t j0, int rows, int cols, int64_t n,
                                                    unsigned long long &cnt, unsigned long long &cs) {
    cnt = 0;
    cs = 0;
    for (int e = threadIdx.x; e < rows * cols; e += NTHREADS) {
        const int64_t i = i0 + e / cols, j = j0 + e % cols;
        if (j < n && i <= j) {
            ++cnt;
            cs += mix64(id_pair_le(uint64_t(i), uint64_t(j), uint64_t(n)));
        }
    }
}

// Statistics slot layout: [slot * kSlotStride + {0: elements, 1: checksum, 2: mapped blocks}]
__device__ __forceinline__ void stats_add(unsigned long long *slots, uint64_t blk, uint64_t elems,
                                          uint64_t csum) {
    unsigned long long *s = slots + (blk % kSlots) * kSlotStride;
    atomicAdd(s + 0, (unsigned long long)elems);
    atomicAdd(s + 1, (unsigned long long)csum);
    atomicAdd(s + 2, 1ull);
}

}  // namespace smx
