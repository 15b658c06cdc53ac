// 4-point contacts on the 4-simplex: the number of quadruplets i < j < k < l
// whose six pairs all lie within a contact radius (the 4-cliques of the
// contact graph) -- a 4-body count over the discrete orthogonal 4-simplex
// (paper Sec. I lists correlation counts among simplex-shaped problems; the
// 4-simplex parallel space is the lambda4 map built on the recursive set of
// Sec. III-D).
//
// Two passes, both over simplex tiles of 64 elements per dimension:
//   1. contact words (2-simplex, one 64-thread block per tile (X, Y), X <= Y):
//      W[Y][64 X + p] bit q = contact(i, j), i = 64 X + p < j = 64 Y + q < n,
//      decided on the FP32 squared distance fl(fma(dz,dz, fma(dy,dy, dx*dx))),
//      d* = fl(x_j* - x_i*), below fl(rc*rc).  Column-tile-major, so the 64
//      words of one tile pair are contiguous.
//   2. cliques (4-simplex, tiles X1 <= X2 <= X3 <= X4, each counted by one
//      wave): lane p1 holds words p1 of the six 64-word blocks of the tile's
//      index sets, and for every contact (p1, p2) and every common neighbour p3
//      (bits of W13[p1] & W23[p2]) adds popcount(W14[p1] & W24[p2] & W34[p3]).
//      The ordering i < j < k < l within equal tiles and the bound n are
//      already in the words.
// Contacts are sparse, so a tile needs little arithmetic: the pass is bound by
// each wave's chain of per-tile word loads (3 KB per tile, from L2) and LDS
// exchange.
#include "smx_device.h"
#include "smx_internal.h"

namespace smx {

constexpr int kQuadWordThreads = 64;
constexpr int kQuadThreads = 256;

template <int MAP>
__global__ __launch_bounds__(kQuadWordThreads) void contact_words_kernel(MapGeom g, const float *__restrict__ Xp,
                                                                        int64_t n, int64_t ldx, float rc2,
                                                                        uint64_t *__restrict__ W, int64_t npad) {
    uint64_t lin;
    int TX, TY;
    if (!tile2_of<MAP, true>(g, lin, TX, TY)) return;
    __shared__ float4 Pc[kQuadTile];
    const int p = threadIdx.x;
    const int64_t i = int64_t(TX) * kQuadTile + p, jc = int64_t(TY) * kQuadTile + p;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (jc < n) v = make_float4(Xp[jc * ldx + 0], Xp[jc * ldx + 1], Xp[jc * ldx + 2], 0.f);
    Pc[p] = v;
    float xi = 0.f, yi = 0.f, zi = 0.f;
    if (i < n) {
        xi = Xp[i * ldx + 0];
        yi = Xp[i * ldx + 1];
        zi = Xp[i * ldx + 2];
    }
    __syncthreads();
    uint64_t word = 0;
    if (i < n) {
        const int64_t jbase = int64_t(TY) * kQuadTile;
        const int q0 = TX == TY ? p + 1 : 0;
        for (int q = q0; q < kQuadTile; ++q) {
            const float4 c = Pc[q];
            const float dx = c.x - xi, dy = c.y - yi, dz = c.z - zi;
            const float s = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
            if (jbase + q < n && s < rc2) word |= uint64_t(1) << q;
        }
    }
    W[int64_t(TY) * npad + i] = word;
}

// Quadruplets i < j < k < l of a 4-simplex tile, in closed form (edge lengths
// below n; runs of equal tile coordinates hold C(t, r) strict r-tuples).
__device__ __forceinline__ uint64_t quad_tile_volume(const int T[4], int64_t n) {
    uint64_t cnt = 1;
    int d = 0;
    while (d < 4) {
        int r = 1;
        while (d + r < 4 && T[d + r] == T[d]) ++r;
        const int64_t rem = n - int64_t(T[d]) * kQuadTile;
        const uint64_t t = rem <= 0 ? 0 : (rem < kQuadTile ? uint64_t(rem) : uint64_t(kQuadTile));
        uint64_t v = 1;
        for (int q = 0; q < r; ++q) v = t < uint64_t(q) ? 0 : v * (t - uint64_t(q)) / uint64_t(q + 1);
        cnt *= v;
        d += r;
    }
    return cnt;
}

// One wave per 64 logical block ids, one tile at a time.  Lane q evaluates the
// map for id 64 (4 b + w) + q, so a wave decodes its 64 ids in one pass and an
// id outside the simplex costs one lane of that pass; the wave then walks the
// mapped tiles (a ballot of the lanes' results) with each tile's coordinates
// read from the lane that decoded it, loading the next tile's words while it
// counts the current one.  Per tile, lane p holds word p of the six 64-word
// blocks of the index sets, keeps its own three in registers, shares the other
// three through the wave's 1.5 KB of LDS, and walks its 64 p2 bits.  A launch
// has G / 256 hardware blocks.
template <int MAP, bool STATS>
__global__ __launch_bounds__(kQuadThreads) void quad_kernel(MapGeom g, const uint64_t *__restrict__ W, int64_t npad,
                                                           int64_t n, unsigned long long *cslots,
                                                           unsigned long long *sslots) {
    // pair sets s = (a, b): 0 (0,1), 1 (0,2), 2 (0,3), 3 (1,2), 4 (1,3), 5 (2,3);
    // sets 3..5 are read across lanes
    __shared__ uint64_t A[kQuadThreads / kWave][3][kQuadTile];
    const int w = threadIdx.x / kWave, p = threadIdx.x & (kWave - 1);
    const uint64_t b = uint64_t(blockIdx.y) * gridDim.x + blockIdx.x;
    const uint64_t base = (b * (kQuadThreads / kWave) + uint64_t(w)) * kWave;
    uint64_t (*Aw)[kQuadTile] = A[w];

    uint64_t mylin = 0;
    int Tq[4] = {0, 0, 0, 0};
    bool ok = false;
    if (base + uint64_t(p) < g.G) ok = tile4_of_id<MAP>(g, uint32_t(base + uint64_t(p)), mylin, Tq);
    uint64_t mask = __ballot(ok);

    // coordinates of the tile decoded by lane q (q uniform), and its words
    auto coords = [&](int q, int T[4]) {
#pragma unroll
        for (int d = 0; d < 4; ++d) T[d] = __builtin_amdgcn_readlane(Tq[d], q);
    };
    auto load = [&](const int T[4], uint64_t a[6]) {
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const int64_t ra = s < 3 ? T[0] : (s < 5 ? T[1] : T[2]);
            const int64_t cb = s == 0 ? T[1] : (s == 1 || s == 3) ? T[2] : T[3];
            a[s] = W[cb * npad + ra * kQuadTile + p];
        }
    };

    uint32_t cnt = 0;
    if (mask != 0) {
        int q = __builtin_ctzll(mask);
        mask &= mask - 1;
        int T[4];
        uint64_t a[6];
        coords(q, T);
        load(T, a);
        while (true) {
            const bool more = mask != 0;
            int qn = 0, Tn[4] = {0, 0, 0, 0};
            uint64_t an[6] = {0, 0, 0, 0, 0, 0};
            if (more) {
                qn = __builtin_ctzll(mask);
                mask &= mask - 1;
                coords(qn, Tn);
                load(Tn, an);
            }
            // the previous tile's reads of this wave's LDS are done before it is
            // overwritten, and the writes land before other lanes read them
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int s = 0; s < 3; ++s) Aw[s][p] = a[3 + s];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            uint64_t bits = a[0];
            while (bits != 0) {
                const int p2 = __builtin_ctzll(bits);
                bits &= bits - 1;
                uint64_t m3 = a[1] & Aw[0][p2];
                const uint64_t wv = a[2] & Aw[1][p2];
                while (m3 != 0) {
                    const int p3 = __builtin_ctzll(m3);
                    m3 &= m3 - 1;
                    cnt += uint32_t(__builtin_popcountll(wv & Aw[2][p3]));
                }
            }
            if (STATS && p == 0) {
                const uint64_t lin = uint64_t(__builtin_amdgcn_readlane(uint32_t(mylin), q)) |
                                     (uint64_t(__builtin_amdgcn_readlane(uint32_t(mylin >> 32), q)) << 32);
                stats_add(sslots, lin, quad_tile_volume(T, n), 0);
            }
            if (!more) break;
            q = qn;
#pragma unroll
            for (int d = 0; d < 4; ++d) T[d] = Tn[d];
#pragma unroll
            for (int s = 0; s < 6; ++s) a[s] = an[s];
        }
    }
    const unsigned c = wave_sum(cnt);
    if (p == 0 && c != 0) atomicAdd(cslots + (base / kWave % kSlots) * kSlotStride, (unsigned long long)c);
}

__global__ void count_finalize_kernel(const unsigned long long *slots, int64_t *out) {
    __shared__ unsigned long long red[kSlots / kWave];
    const unsigned long long v = block_sum<unsigned long long, kSlots>(slots[threadIdx.x * kSlotStride], red);
    if (threadIdx.x == 0) out[0] = int64_t(v);
}

int launch_contact_words(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float rc2, uint64_t *W,
                         int64_t npad, hipStream_t s) {
    prof_begin(K_QUAD_WORDS, s);
    for_each_launch(g, [&](auto M, const MapGeom &gg) {
        constexpr int MAPK = decltype(M)::value;
        const dim3 grid = MAPK == MAP_BBOX ? dim3(gg.nb, gg.nb, 1) : grid_for(gg.G, kQuadWordThreads);
        hipLaunchKernelGGL((contact_words_kernel<MAPK>), grid, dim3(kQuadWordThreads), 0, s, gg, X, n, ldx, rc2, W,
                           npad);
    });
    prof_end(K_QUAD_WORDS, s);
    return check_launch("contact words");
}

int launch_quad(const MapGeom &g, const uint64_t *W, int64_t npad, int64_t n, unsigned long long *cslots,
                unsigned long long *sslots, hipStream_t s) {
    prof_begin(K_QUAD, s);
    for_each_launch(g, [&](auto M, const MapGeom &gg) {
        constexpr int MAPK = decltype(M)::value;
        const uint64_t per_block = kQuadThreads;  // one id per thread
        const dim3 grid = grid_for((gg.G + per_block - 1) / per_block, kQuadThreads);
        if (sslots)
            hipLaunchKernelGGL((quad_kernel<MAPK, true>), grid, dim3(kQuadThreads), 0, s, gg, W, npad, n, cslots,
                               sslots);
        else
            hipLaunchKernelGGL((quad_kernel<MAPK, false>), grid, dim3(kQuadThreads), 0, s, gg, W, npad, n, cslots,
                               sslots);
    });
    prof_end(K_QUAD, s);
    return check_launch("quad contacts");
}

int launch_count_finalize(const unsigned long long *slots, int64_t *out, hipStream_t s) {
    prof_begin(K_FINALIZE, s);
    hipLaunchKernelGGL(count_finalize_kernel, dim3(1), dim3(kSlots), 0, s, slots, out);
    prof_end(K_FINALIZE, s);
    return check_launch("count finalize");
}

SMX_CHECK_READER(check_flags_quad)

}  // namespace smx
