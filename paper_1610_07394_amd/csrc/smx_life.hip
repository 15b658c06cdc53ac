// Conway's Life on the discrete orthogonal 2-simplex of cells (i, j),
// 0 <= i <= j < n: a cellular automaton on a triangular domain (paper Sec. I),
// one generation per launch, mapped over the 2-simplex of 64 x 64 cell tiles.
// Cells outside the triangle are dead and stay dead; the rule is birth on 3
// live neighbours and survival on 2 or 3 (Moore neighbourhood).
//
// Layout (input and output): tile-contiguous bytes, tile (X, Y), X <= Y < nb =
// ceil(n / 64), at rank (Y(Y+1)/2 + X) * 4096, cell (i, j) at 64 (i mod 64) +
// (j mod 64), 1 = alive; the output holds 0 outside the triangle, and the input
// is not read there.
//
// Block: 256 threads own tile (X, Y).  Thread t holds 16 consecutive cells of
// row t / 4 as four 32-bit words, one byte per cell.  LDS keeps the tile's 64
// rows with the ring rows above and below (rows of 64 bytes: the 16-byte reads
// of a wave touch every bank once) and the left and right ring columns in
// arrays of their own.  The ring comes from the eight neighbouring tiles (those
// outside the simplex of tiles give dead cells): the two columns one byte per
// thread, the two rows as 16-byte words.
//
// Neighbour counts are byte-parallel: for each of the three rows a word plus
// its two one-byte shifts (the shifted-in bytes from the adjacent word or the
// ring) sums three horizontal cells per byte, and the three row sums give the
// 3 x 3 total T <= 9 per byte without carries.  A cell lives iff T = 3, or T = 4
// and it was alive; a byte equals v iff bit 7 of 0x80 - (T xor v) is set, which
// for bytes below 0x80 borrows from no other byte.
#include "smx_device.h"
#include "smx_internal.h"

namespace smx {

constexpr int kLifeThreads = 256;
constexpr int kLifeRow = kLifeTile;  // LDS row stride: 64 cells

__device__ __forceinline__ uint64_t life_offset(int64_t i, int64_t j) {
    const uint64_t ti = uint64_t(i) >> 6, tj = uint64_t(j) >> 6;
    return (tj * (tj + 1) / 2 + ti) * 4096 + uint64_t(i & 63) * 64 + uint64_t(j & 63);
}

// Clear the bytes of cells (i, jb .. jb + 15) outside the triangle 0 <= i <= j < n.
__device__ __forceinline__ uint4 life_mask16(uint4 w, int64_t i, int64_t jb, int64_t n) {
    uint32_t q[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const int64_t j = jb + c;
        if (!(i >= 0 && i <= j && j < n)) q[c >> 2] &= ~(0xFFu << (8 * (c & 3)));
    }
    return make_uint4(q[0], q[1], q[2], q[3]);
}

// bit 7 of each byte set where the byte of T equals the matching byte of v
// (all bytes of T and v below 0x80)
__device__ __forceinline__ uint32_t bytes_eq(uint32_t T, uint32_t v) {
    return (0x80808080u - (T ^ v)) & 0x80808080u;
}

template <int MAP, bool STATS>
__global__ __launch_bounds__(kLifeThreads) void life_kernel(MapGeom g, const uint8_t *__restrict__ S,
                                                            uint8_t *__restrict__ D, int64_t n,
                                                            unsigned long long *slots) {
    uint64_t lin;
    int X, Y;
    // No XCD renumbering: the map hands consecutive blocks consecutive tiles of
    // one tile column, and the tiles left and right of a tile one parallel-space
    // row apart, a multiple of 8 blocks, so the default round-robin places them on
    // the same XCD a few dozen blocks apart, where the ring columns hit its L2.
    if (!tile2_of<MAP, false>(g, lin, X, Y)) return;
    __shared__ __attribute__((aligned(16))) uint8_t H[(kLifeTile + 2) * kLifeRow];
    __shared__ uint8_t Lc[kLifeTile + 2], Rc[kLifeTile + 2];
    __shared__ unsigned long long red[kLifeThreads / kWave];
    const int t = threadIdx.x;
    const int64_t i0 = int64_t(X) * kLifeTile, j0 = int64_t(Y) * kLifeTile;
    const uint64_t base = (uint64_t(Y) * (Y + 1) / 2 + uint64_t(X)) * 4096;
    const int r = t >> 2, k = t & 3, c0 = k << 4;
    // tiles that reach the diagonal or n: cells outside the triangle read as dead
    // whatever the buffer holds there, and are written as 0
    const bool edge = X == Y || j0 + kLifeTile > n;

    // ring loads first, so that their latency overlaps the tile's:
    // threads 0..65 the left column (j0 - 1), 66..131 the right one (j0 + 64),
    // rows i0 - 1 .. i0 + 64; threads 132..139 the rows above and below, 16 cells each
    uint8_t cv = 0;
    uint4 rv = make_uint4(0, 0, 0, 0);
    if (t < 2 * (kLifeTile + 2)) {
        const int hr = t < kLifeTile + 2 ? t : t - (kLifeTile + 2);
        const int64_t i = i0 - 1 + hr, j = t < kLifeTile + 2 ? j0 - 1 : j0 + kLifeTile;
        if (i >= 0 && i <= j && j < n) cv = S[life_offset(i, j)];
    } else if (t < 2 * (kLifeTile + 2) + 8) {
        const int u = t - 2 * (kLifeTile + 2);
        const int64_t i = u < 4 ? i0 - 1 : i0 + kLifeTile, jb = j0 + 16 * (u & 3);
        // the 16 cells lie in one row of tile (i / 64, Y); fetched if any is inside
        if (i >= 0 && i <= jb + 15 && jb < n)
            rv = life_mask16(*reinterpret_cast<const uint4 *>(S + life_offset(i, jb)), i, jb, n);
    }
    uint4 w = *reinterpret_cast<const uint4 *>(S + base + r * 64 + c0);
    if (edge) w = life_mask16(w, i0 + r, j0 + c0, n);
    *reinterpret_cast<uint4 *>(&H[(r + 1) * kLifeRow + c0]) = w;
    if (t < kLifeTile + 2) {
        Lc[t] = cv;
    } else if (t < 2 * (kLifeTile + 2)) {
        Rc[t - (kLifeTile + 2)] = cv;
    } else if (t < 2 * (kLifeTile + 2) + 8) {
        const int u = t - 2 * (kLifeTile + 2);
        *reinterpret_cast<uint4 *>(&H[(u < 4 ? 0 : kLifeTile + 1) * kLifeRow + 16 * (u & 3)]) = rv;
    }
    __syncthreads();

    // 3 x 3 totals per byte over LDS rows r, r + 1, r + 2 (cell rows i0 + r - 1 .. i0 + r + 1)
    uint32_t T[4] = {0u, 0u, 0u, 0u}, M[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int R = r + d;
        const uint4 v = *reinterpret_cast<const uint4 *>(&H[R * kLifeRow + c0]);
        const uint32_t lb = k == 0 ? uint32_t(Lc[R]) : uint32_t(H[R * kLifeRow + c0 - 1]);
        const uint32_t rb = k == 3 ? uint32_t(Rc[R]) : uint32_t(H[R * kLifeRow + c0 + 16]);
        const uint32_t q[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t lo = e == 0 ? (lb << 24) : q[e - 1];
            const uint32_t hi = e == 3 ? rb : q[e + 1];
            // cells c - 1 and c + 1 moved into the byte of cell c
            const uint32_t left = __builtin_amdgcn_alignbyte(q[e], lo, 3);
            const uint32_t right = __builtin_amdgcn_alignbyte(hi, q[e], 1);
            T[e] += left + q[e] + right;
            if (d == 1) M[e] = q[e];
        }
    }
    uint32_t o[4];
    unsigned alive_count = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const uint32_t live = bytes_eq(T[e], 0x03030303u) | (bytes_eq(T[e], 0x04040404u) & (M[e] << 7));
        o[e] = live >> 7;
    }
    uint4 out = make_uint4(o[0], o[1], o[2], o[3]);
    if (edge) out = life_mask16(out, i0 + r, j0 + c0, n);
    // the new generation is not read again by this launch: a streaming
    // (non-temporal) store keeps the L2 for the ring cells the neighbouring
    // tiles read (measured 0.254 -> 0.244 ms per generation at n = 32768)
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 ov = {out.x, out.y, out.z, out.w};
    __builtin_nontemporal_store(ov, reinterpret_cast<u32x4 *>(D + base + r * 64 + c0));
    if (STATS) {
        alive_count = __builtin_popcount(out.x) + __builtin_popcount(out.y) + __builtin_popcount(out.z) +
                      __builtin_popcount(out.w);
        const unsigned long long a = block_sum<unsigned long long, kLifeThreads>(alive_count, red);
        if (t == 0) stats_add(slots, lin, a, 0);
    }
}

template <int MAP>
static void go_life(const MapGeom &g, const uint8_t *S, uint8_t *D, int64_t n, unsigned long long *slots,
                    hipStream_t s) {
    const dim3 grid = MAP == MAP_BBOX ? dim3(g.nb, g.nb, 1) : grid_for(g.G, kLifeThreads);
    if (slots)
        hipLaunchKernelGGL((life_kernel<MAP, true>), grid, dim3(kLifeThreads), 0, s, g, S, D, n, slots);
    else
        hipLaunchKernelGGL((life_kernel<MAP, false>), grid, dim3(kLifeThreads), 0, s, g, S, D, n, slots);
}

int launch_life(const MapGeom &g, const uint8_t *S, uint8_t *D, int64_t n, unsigned long long *slots,
                hipStream_t s) {
    prof_begin(K_LIFE, s);
    for_each_launch(g, [&](auto M, const MapGeom &gg) { go_life<decltype(M)::value>(gg, S, D, n, slots, s); });
    prof_end(K_LIFE, s);
    return check_launch("simplex life");
}

SMX_CHECK_READER(check_flags_life)

}  // namespace smx
