// Map-dump kernels: every launched block evaluates its map once (block
// uniform, scalar unit), records its tile, and visits the elements of the tile
// under the simplex mask, counting them and summing SplitMix64 of their ids.
// This is the map with an almost empty body: it isolates the cost of the map
// and of the blocks a map wastes (paper Sec. I and III).  The count kernels
// keep one block per tile with a closed-form count; the decode kernel drops
// the block per tile and evaluates the map once per lane.
#include "smx_device.h"
#include "smx_internal.h"

namespace smx {

constexpr int kMapThreads = 256;

__global__ void fill_u64_kernel(uint64_t *p, size_t count) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

int launch_fill_u64(uint64_t *p, size_t count, hipStream_t s) {
    if (count == 0) return SMX_OK;
    const unsigned blocks = unsigned((count + 255) / 256);
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks), dim3(256), 0, s, p, count);
    return check_launch("fill");
}

__global__ void stats_finalize_kernel(const unsigned long long *slots, uint64_t launched,
                                      int64_t *out) {
    __shared__ unsigned long long red[3][kSlots / kWave];
    const int t = threadIdx.x;  // kSlots threads
    unsigned long long v[3];
    for (int c = 0; c < 3; ++c) v[c] = wave_sum(slots[t * kSlotStride + c]);
    if ((t & (kWave - 1)) == 0)
        for (int c = 0; c < 3; ++c) red[c][t / kWave] = v[c];
    __syncthreads();
    if (t == 0) {
        for (int c = 0; c < 3; ++c) {
            unsigned long long r = 0;
            for (int w = 0; w < kSlots / kWave; ++w) r += red[c][w];
            out[c] = int64_t(r);
        }
        out[3] = int64_t(launched);
    }
}

int launch_stats_finalize(const unsigned long long *slots, uint64_t launched, int64_t *d_stats,
                          hipStream_t s) {
    prof_begin(K_FINALIZE, s);
    hipLaunchKernelGGL(stats_finalize_kernel, dim3(1), dim3(kSlots), 0, s, slots, launched,
                       d_stats);
    prof_end(K_FINALIZE, s);
    return check_launch("stats finalize");
}

template <int MAP, bool STRICT>
__global__ __launch_bounds__(kMapThreads) void map2_kernel(MapGeom g, int64_t n, int rho, int lgrho,
                                                          int32_t *tiles, unsigned long long *slots) {
    uint64_t lin;
    int X = -1, Y = -1;
    const bool ok = tile2_of<MAP, false>(g, lin, X, Y);
    if (launch_tail<MAP>(g)) return;
    if (tiles != nullptr && threadIdx.x == 0) {
        tiles[2 * lin + 0] = ok ? X : -1;
        tiles[2 * lin + 1] = ok ? Y : -1;
    }
    if (!ok || slots == nullptr) return;
    __shared__ unsigned long long red[2][kMapThreads / kWave];
    unsigned long long cnt = 0, cs = 0;
    const int64_t i0 = int64_t(X) * rho, j0 = int64_t(Y) * rho;
    const int rmask = rho - 1;
    for (int e = threadIdx.x; e < rho * rho; e += kMapThreads) {
        const int64_t i = i0 + (e >> lgrho), j = j0 + (e & rmask);
        const bool v = j < n && (STRICT ? i < j : i <= j);
        if (v) {
            ++cnt;
            cs += mix64(STRICT ? id_pair_lt(i, j) : id_pair_le(i, j, uint64_t(n)));
        }
    }
    const unsigned long long c = block_sum<unsigned long long, kMapThreads>(cnt, red[0]);
    const unsigned long long h = block_sum<unsigned long long, kMapThreads>(cs, red[1]);
    if (threadIdx.x == 0) stats_add(slots, lin, c, h);
}

template <int MAP, bool STRICT>
__global__ __launch_bounds__(kMapThreads) void map3_kernel(MapGeom g, int64_t n, int rho, int lgrho,
                                                          int32_t *tiles, unsigned long long *slots) {
    uint64_t lin;
    int X = -1, Y = -1, Z = -1;
    const bool ok = tile3_of<MAP, false>(g, lin, X, Y, Z);
    if (launch_tail<MAP>(g)) return;
    if (tiles != nullptr && threadIdx.x == 0) {
        tiles[3 * lin + 0] = ok ? X : -1;
        tiles[3 * lin + 1] = ok ? Y : -1;
        tiles[3 * lin + 2] = ok ? Z : -1;
    }
    if (!ok || slots == nullptr) return;
    __shared__ unsigned long long red[2][kMapThreads / kWave];
    unsigned long long cnt = 0, cs = 0;
    const int64_t i0 = int64_t(X) * rho, j0 = int64_t(Y) * rho, k0 = int64_t(Z) * rho;
    const int rmask = rho - 1;
    for (int e = threadIdx.x; e < rho * rho * rho; e += kMapThreads) {
        const int64_t i = i0 + (e >> (2 * lgrho)), j = j0 + ((e >> lgrho) & rmask), k = k0 + (e & rmask);
        const bool v = k < n && (STRICT ? (i < j && j < k) : (i <= j && j <= k));
        if (v) {
            ++cnt;
            cs += mix64(STRICT ? id_trip_lt(i, j, k) : id_trip_le(i, j, k));
        }
    }
    const unsigned long long c = block_sum<unsigned long long, kMapThreads>(cnt, red[0]);
    const unsigned long long h = block_sum<unsigned long long, kMapThreads>(cs, red[1]);
    if (threadIdx.x == 0) stats_add(slots, lin, c, h);
}

template <int MAP, bool STRICT>
__global__ __launch_bounds__(kMapThreads) void map4_kernel(MapGeom g, int64_t n, int rho, int lgrho,
                                                          int32_t *tiles, unsigned long long *slots) {
    uint64_t lin;
    int X[4] = {-1, -1, -1, -1};
    const bool ok = tile4_of<MAP, false>(g, lin, X);
    if (launch_tail<MAP_LINEAR>(g)) return;  // every m = 4 map runs on a 1-D / 2-D launch
    if (tiles != nullptr && threadIdx.x == 0) {
        for (int d = 0; d < 4; ++d) tiles[4 * lin + d] = ok ? X[d] : -1;
    }
    if (!ok || slots == nullptr) return;
    __shared__ unsigned long long red[2][kMapThreads / kWave];
    unsigned long long cnt = 0, cs = 0;
    const int64_t i0 = int64_t(X[0]) * rho, j0 = int64_t(X[1]) * rho, k0 = int64_t(X[2]) * rho,
                  l0 = int64_t(X[3]) * rho;
    const int rmask = rho - 1;
    for (int e = threadIdx.x; e < rho * rho * rho * rho; e += kMapThreads) {
        const int64_t i = i0 + (e >> (3 * lgrho)), j = j0 + ((e >> (2 * lgrho)) & rmask),
                      k = k0 + ((e >> lgrho) & rmask), l = l0 + (e & rmask);
        const bool v = l < n && (STRICT ? (i < j && j < k && k < l) : (i <= j && j <= k && k <= l));
        if (v) {
            ++cnt;
            cs += mix64(STRICT ? id_quad_lt(i, j, k, l) : id_quad_le(i, j, k, l));
        }
    }
    const unsigned long long c = block_sum<unsigned long long, kMapThreads>(cnt, red[0]);
    const unsigned long long h = block_sum<unsigned long long, kMapThreads>(cs, red[1]);
    if (threadIdx.x == 0) stats_add(slots, lin, c, h);
}

// Element count of one tile in closed form: t = elements of a tile edge that
// lie below n; a diagonal pair of tile coordinates holds a triangle, a
// diagonal triple a tetrahedron.
__device__ __forceinline__ uint64_t edge_len(int T, int rho, int64_t n) {
    const int64_t r = n - int64_t(T) * rho;
    return r <= 0 ? 0 : (r < rho ? uint64_t(r) : uint64_t(rho));
}
__device__ __forceinline__ uint64_t tri_cnt(uint64_t t, bool strict) {
    return strict ? (t == 0 ? 0 : t * (t - 1) / 2) : t * (t + 1) / 2;
}
__device__ __forceinline__ uint64_t tet_cnt(uint64_t t, bool strict) {
    return strict ? (t < 3 ? 0 : t * (t - 1) * (t - 2) / 6) : t * (t + 1) * (t + 2) / 6;
}

// Map-only parallel space: each mapped block adds its tile's element count
// (one atomic from one lane); no per-element work, so the kernel time is the
// cost of the blocks launched plus one map evaluation per block -- the
// quantity the paper's parallel-space analysis is about.  The block keeps the
// 256 threads of the other kernels, but only its first wave evaluates the map
// (the others have no element work here and leave at once, for every map).
template <int MAP, bool STRICT>
__global__ __launch_bounds__(kMapThreads) void count2_kernel(MapGeom g, int64_t n, int rho,
                                                            unsigned long long *slots) {
    if (threadIdx.x >= kWave) return;
    uint64_t lin;
    int X, Y;
    if (!tile2_of<MAP, false>(g, lin, X, Y)) return;
    if (threadIdx.x != 0) return;
    const uint64_t a = edge_len(X, rho, n), c = edge_len(Y, rho, n);
    const uint64_t cnt = X < Y ? a * c : tri_cnt(a, STRICT);
    unsigned long long *s = slots + (lin % kSlots) * kSlotStride;
    atomicAdd(s + 0, (unsigned long long)cnt);
    atomicAdd(s + 2, 1ull);
}

template <int MAP, bool STRICT>
__global__ __launch_bounds__(kMapThreads) void count3_kernel(MapGeom g, int64_t n, int rho,
                                                            unsigned long long *slots) {
    if (threadIdx.x >= kWave) return;
    uint64_t lin;
    int X, Y, Z;
    if (!tile3_of<MAP, false>(g, lin, X, Y, Z)) return;
    if (threadIdx.x != 0) return;
    const uint64_t a = edge_len(X, rho, n), b = edge_len(Y, rho, n), c = edge_len(Z, rho, n);
    uint64_t cnt;
    if (X < Y && Y < Z) cnt = a * b * c;
    else if (X == Y && Y < Z) cnt = tri_cnt(a, STRICT) * c;
    else if (X < Y) cnt = a * tri_cnt(b, STRICT);
    else cnt = tet_cnt(a, STRICT);
    unsigned long long *s = slots + (lin % kSlots) * kSlotStride;
    atomicAdd(s + 0, (unsigned long long)cnt);
    atomicAdd(s + 2, 1ull);
}

// Elements of a 4-simplex tile: consecutive equal tile coordinates form runs;
// a run of r equal coordinates with edge length t holds C(t + r - 1, r) (or
// C(t, r) strict) sorted r-tuples, and distinct runs multiply.
__device__ __forceinline__ uint64_t run_cnt(uint64_t t, int r, bool strict) {
    uint64_t v = 1;
    for (int q = 0; q < r; ++q) v = v * (strict ? t - uint64_t(q) : t + uint64_t(q)) / uint64_t(q + 1);
    return strict && t < uint64_t(r) ? 0 : v;
}

template <int MAP, bool STRICT>
__global__ __launch_bounds__(kMapThreads) void count4_kernel(MapGeom g, int64_t n, int rho,
                                                            unsigned long long *slots) {
    if (threadIdx.x >= kWave) return;
    uint64_t lin;
    int X[4];
    if (!tile4_of<MAP, false>(g, lin, X)) return;
    if (threadIdx.x != 0) return;
    uint64_t cnt = 1;
    int d = 0;
    while (d < 4) {
        int r = 1;
        while (d + r < 4 && X[d + r] == X[d]) ++r;
        cnt *= run_cnt(edge_len(X[d], rho, n), r, STRICT);
        d += r;
    }
    unsigned long long *s = slots + (lin % kSlots) * kSlotStride;
    atomicAdd(s + 0, (unsigned long long)cnt);
    atomicAdd(s + 2, 1ull);
}

int launch_count(int m, const MapGeom &g, int64_t n, int rho, int map, int strict,
                 unsigned long long *slots, hipStream_t s) {
    const int kid = m == 2 ? K_MAP2 : m == 3 ? K_MAP3 : K_MAP4;
    prof_begin(kid, s);
    (void)map;
    for_each_launch(g, [&](auto M, const MapGeom &g) {
        constexpr int MAPK = decltype(M)::value;
        if (m == 4) {
            const dim3 grid = grid_for(g.G, kMapThreads);
            if (strict) hipLaunchKernelGGL((count4_kernel<MAPK, true>), grid, dim3(kMapThreads), 0, s, g, n, rho, slots);
            else hipLaunchKernelGGL((count4_kernel<MAPK, false>), grid, dim3(kMapThreads), 0, s, g, n, rho, slots);
        } else if (m == 2) {
            const dim3 grid = MAPK == MAP_BBOX ? dim3(g.nb, g.nb, 1) : grid_for(g.G, kMapThreads);
            if (strict) hipLaunchKernelGGL((count2_kernel<MAPK, true>), grid, dim3(kMapThreads), 0, s, g, n, rho, slots);
            else hipLaunchKernelGGL((count2_kernel<MAPK, false>), grid, dim3(kMapThreads), 0, s, g, n, rho, slots);
        } else {
            const dim3 grid = MAPK == MAP_BBOX ? dim3(g.nb, g.nb, g.nb) : grid_for(g.G, kMapThreads);
            if (strict) hipLaunchKernelGGL((count3_kernel<MAPK, true>), grid, dim3(kMapThreads), 0, s, g, n, rho, slots);
            else hipLaunchKernelGGL((count3_kernel<MAPK, false>), grid, dim3(kMapThreads), 0, s, g, n, rho, slots);
        }
    });
    prof_end(kid, s);
    return check_launch("simplex_count");
}

// Lane-parallel decode: every thread evaluates the map for kDecodeIds logical
// block ids (id = 256 (kDecodeIds b + r) + t), so a launch measures the map's
// arithmetic per id, free of block dispatch.  A mapped tile adds 1 to the count
// and SplitMix64 of its colex rank (Y(Y+1)/2 + X, then the tetrahedral and
// pentatope terms) to the checksum: over a bijection onto T_m these sums are
// |T_m| and the checksum of the range [0, |T_m|).
constexpr int kDecodeIds = 16;

__device__ __forceinline__ uint64_t colex_rank(int m, const int T[4]) {
    const uint64_t a = uint64_t(T[0]), b = uint64_t(T[1]), c = uint64_t(T[2]), d = uint64_t(T[3]);
    uint64_t r = a + b * (b + 1) / 2;
    if (m >= 3) r += c * (c + 1) * (c + 2) / 6;
    if (m >= 4) r += d * (d + 1) * (d + 2) * (d + 3) / 24;
    return r;
}

template <int MAP, int M>
__global__ __launch_bounds__(kMapThreads) void decode_kernel(MapGeom g, unsigned long long *slots) {
    __shared__ unsigned long long red[2][kMapThreads / kWave];
    const uint64_t b = uint64_t(blockIdx.y) * gridDim.x + blockIdx.x;
    unsigned long long cnt = 0, cs = 0;
#pragma unroll 4
    for (int r = 0; r < kDecodeIds; ++r) {
        const uint64_t id = (b * kDecodeIds + uint64_t(r)) * kMapThreads + threadIdx.x;
        if (id >= g.G) break;
        uint64_t lin;
        int T[4] = {0, 0, 0, 0};
        bool ok;
        if (M == 2) ok = tile2_of_id<MAP>(g, uint32_t(id), lin, T[0], T[1]);
        else if (M == 3) ok = tile3_of_id<MAP>(g, uint32_t(id), lin, T[0], T[1], T[2]);
        else ok = tile4_of_id<MAP>(g, uint32_t(id), lin, T);
        if (ok) {
            ++cnt;
            cs += mix64(colex_rank(M, T));
        }
    }
    const unsigned long long c = block_sum<unsigned long long, kMapThreads>(cnt, red[0]);
    const unsigned long long h = block_sum<unsigned long long, kMapThreads>(cs, red[1]);
    if (threadIdx.x == 0 && c != 0) {
        unsigned long long *sl = slots + (b % kSlots) * kSlotStride;
        atomicAdd(sl + 0, c);
        atomicAdd(sl + 1, h);
        atomicAdd(sl + 2, 1ull);
    }
}

int launch_decode(int m, const MapGeom &g, unsigned long long *slots, hipStream_t s) {
    prof_begin(K_DECODE, s);
    for_each_launch(g, [&](auto Mk, const MapGeom &gg) {
        constexpr int MAPK = decltype(Mk)::value;
        const uint64_t per_block = uint64_t(kMapThreads) * kDecodeIds;
        const dim3 grid = grid_for((gg.G + per_block - 1) / per_block, kMapThreads);
        if (m == 2) hipLaunchKernelGGL((decode_kernel<MAPK, 2>), grid, dim3(kMapThreads), 0, s, gg, slots);
        else if (m == 3) hipLaunchKernelGGL((decode_kernel<MAPK, 3>), grid, dim3(kMapThreads), 0, s, gg, slots);
        else hipLaunchKernelGGL((decode_kernel<MAPK, 4>), grid, dim3(kMapThreads), 0, s, gg, slots);
    });
    prof_end(K_DECODE, s);
    return check_launch("simplex decode");
}

template <int MAP>
static void go_map2(const MapGeom &g, int64_t n, int rho, int lgrho, int strict, int32_t *tiles,
                    unsigned long long *slots, hipStream_t s) {
    const dim3 grid = MAP == MAP_BBOX ? dim3(g.nb, g.nb, 1) : grid_for(g.G, kMapThreads);
    if (strict)
        hipLaunchKernelGGL((map2_kernel<MAP, true>), grid, dim3(kMapThreads), 0, s, g, n, rho, lgrho,
                           tiles, slots);
    else
        hipLaunchKernelGGL((map2_kernel<MAP, false>), grid, dim3(kMapThreads), 0, s, g, n, rho, lgrho,
                           tiles, slots);
}

template <int MAP>
static void go_map3(const MapGeom &g, int64_t n, int rho, int lgrho, int strict, int32_t *tiles,
                    unsigned long long *slots, hipStream_t s) {
    const dim3 grid = MAP == MAP_BBOX ? dim3(g.nb, g.nb, g.nb) : grid_for(g.G, kMapThreads);
    if (strict)
        hipLaunchKernelGGL((map3_kernel<MAP, true>), grid, dim3(kMapThreads), 0, s, g, n, rho, lgrho,
                           tiles, slots);
    else
        hipLaunchKernelGGL((map3_kernel<MAP, false>), grid, dim3(kMapThreads), 0, s, g, n, rho, lgrho,
                           tiles, slots);
}

template <int MAP>
static void go_map4(const MapGeom &g, int64_t n, int rho, int lgrho, int strict, int32_t *tiles,
                    unsigned long long *slots, hipStream_t s) {
    const dim3 grid = grid_for(g.G, kMapThreads);
    if (strict)
        hipLaunchKernelGGL((map4_kernel<MAP, true>), grid, dim3(kMapThreads), 0, s, g, n, rho, lgrho,
                           tiles, slots);
    else
        hipLaunchKernelGGL((map4_kernel<MAP, false>), grid, dim3(kMapThreads), 0, s, g, n, rho, lgrho,
                           tiles, slots);
}

int launch_map4(const MapGeom &g, int64_t n, int rho, int strict, int32_t *tiles,
                unsigned long long *slots, hipStream_t s) {
    const int lgrho = floor_log2_u32(uint32_t(rho));
    prof_begin(K_MAP4, s);
    for_each_launch(g, [&](auto M, const MapGeom &gg) { go_map4<decltype(M)::value>(gg, n, rho, lgrho, strict, tiles, slots, s); });
    prof_end(K_MAP4, s);
    return check_launch("simplex_map4");
}

int launch_map2(const MapGeom &g, int64_t n, int rho, int map, int strict, int32_t *tiles,
                unsigned long long *slots, hipStream_t s) {
    const int lgrho = floor_log2_u32(uint32_t(rho));
    prof_begin(K_MAP2, s);
    (void)map;
    for_each_launch(g, [&](auto M, const MapGeom &gg) { go_map2<decltype(M)::value>(gg, n, rho, lgrho, strict, tiles, slots, s); });
    prof_end(K_MAP2, s);
    return check_launch("simplex_map2");
}

int launch_map3(const MapGeom &g, int64_t n, int rho, int map, int strict, int32_t *tiles,
                unsigned long long *slots, hipStream_t s) {
    const int lgrho = floor_log2_u32(uint32_t(rho));
    prof_begin(K_MAP3, s);
    (void)map;
    for_each_launch(g, [&](auto M, const MapGeom &gg) { go_map3<decltype(M)::value>(gg, n, rho, lgrho, strict, tiles, slots, s); });
    prof_end(K_MAP3, s);
    return check_launch("simplex_map3");
}

SMX_CHECK_READER(check_flags_map)

}  // namespace smx
