// Packed Euclidean distance matrix, Gram form on the BF16 matrix cores.
//
//   D_ij = |x_i|^2 + |x_j|^2 - 2 G_ij,  G = X X^T on the tile pair (I, J),
//
// with G from v_mfma_f32_32x32x16_bf16 (FP32 accumulation) and the norms in
// FP32 from the FP32 input.  Plain BF16: G = hi hi^T.  Split BF16 (hi =
// bf16(x), lo = bf16(x - hi), both round-to-nearest-even): G = hi hi^T +
// hi lo^T + lo hi^T, dropping lo lo^T (relative size 2^-16).  D is clamped
// at 0 and the diagonal is set to exactly 0 (the Gram form cancels there).
//
// Block: 256 threads (4 waves as 2 x 2), tile T x T of the packed upper
// triangle (T = 256 for n >= 16384, else 128), each wave T/2 x T/2 in MFMA
// tiles of 32 x 32.  K advances in
// chunks of 32 BF16 through two alternating LDS buffers filled directly from
// global memory in MFMA fragment order (see the staging notes below), so the
// loads of chunk s + 1 are in flight while the matrix cores run chunk s.
#include "smx_device.h"
#include "smx_internal.h"

namespace smx {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

constexpr int kGramThreads = 256;

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// Operand layout in HBM ("fragment order").  hi and lo are stored as 1 KB
// blocks, one per (32-row block rb, 16-wide k block kb), at uint4 index
// (rb * KB + kb) * 64 + s, KB = dpad / 16, where slot s holds row
// 32 rb + (s & 31), k = 16 kb + 8 (s >> 5) .. +7: exactly the operand a lane
// s of v_mfma_f32_32x32x16_bf16 reads.  So a staging load is one contiguous
// 1 KB run.  Rows are padded with zeros to npad = 32 ceil(n / 32), k to dpad.
//
// One wave per row: each lane converts 8 consecutive k (one 16-byte slot of
// hi and of lo) and adds their squares to an FP32 norm (lane-ordered FMA
// sums, then a fixed wave tree).
__global__ __launch_bounds__(256) void gram_prep_kernel(const float *__restrict__ X, int64_t n,
                                                        int64_t d, int64_t ldx, int64_t dpad,
                                                        int64_t npad, uint4 *__restrict__ hi,
                                                        uint4 *__restrict__ lo,
                                                        float *__restrict__ norms) {
    const int lane = threadIdx.x & 63;
    const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (row >= npad) return;
    const int64_t KB = dpad / 16;
    float acc = 0.f;
    for (int64_t q = lane; q < dpad / 8; q += 64) {
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t k = 8 * q + e;
            x[e] = (row < n && k < d) ? X[row * ldx + k] : 0.f;
            acc = __builtin_fmaf(x[e], x[e], acc);
        }
        uint32_t h[4], l[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint16_t h0 = bf16_rne(x[2 * e]), h1 = bf16_rne(x[2 * e + 1]);
            h[e] = uint32_t(h0) | (uint32_t(h1) << 16);
            const uint16_t l0 = bf16_rne(x[2 * e] - bf16_to_f32(h0));
            const uint16_t l1 = bf16_rne(x[2 * e + 1] - bf16_to_f32(h1));
            l[e] = uint32_t(l0) | (uint32_t(l1) << 16);
        }
        const int64_t slot = ((row >> 5) * KB + (q >> 1)) * 64 + (row & 31) + 32 * (q & 1);
        hi[slot] = make_uint4(h[0], h[1], h[2], h[3]);
        if (lo != nullptr) lo[slot] = make_uint4(l[0], l[1], l[2], l[3]);
    }
    acc = wave_sum(acc);
    if (lane == 0 && row < n) norms[row] = acc;
}

int launch_gram_prep(const float *X, int64_t n, int64_t d, int64_t ldx, int64_t dpad, uint16_t *hi,
                     uint16_t *lo, float *norms, bool split, hipStream_t s) {
    const int64_t npad = gram_rows(n);
    prof_begin(K_GRAM_PREP, s);
    hipLaunchKernelGGL(gram_prep_kernel, dim3(uint32_t(npad / 4)), dim3(256), 0, s, X, n, d, ldx, dpad,
                       npad, reinterpret_cast<uint4 *>(hi), split ? reinterpret_cast<uint4 *>(lo) : nullptr,
                       norms);
    prof_end(K_GRAM_PREP, s);
    return check_launch("gram prep");
}

// Staging.  Every MFMA operand fragment travels from global memory straight
// into LDS with global_load_lds_dwordx4: one wave load moves one contiguous
// 1 KB block of the fragment-ordered operand, lane s writing the 16 bytes it
// later reads back as its operand.  Block (mb, ks) of a T-row panel chunk
// holds rows mb*32 + (s & 31), k = ks*16 + 8*(s >> 5) .. +7, so an operand
// read is base + 16*lane (no bank conflicts) and staging costs no VGPRs.  Two LDS buffers alternate: a wave
// reads the fragments of chunk s, issues the loads of chunk s + 1 into the
// other buffer, then runs the MFMAs of chunk s while those loads are in flight.
//
// WT = wave tile (64 or 128): the block tile is T = 2 WT, each wave owns
// WT / 32 x WT / 32 MFMA tiles.  T = 256 halves the operand bytes per flop
// (split BF16: 4 operand arrays x 16 KB per chunk, 128 KB of LDS, one block
// per CU with 256 accumulator registers per lane).
template <bool SPLIT, int WT>
struct GramCfg {
    static constexpr int NARR = SPLIT ? 4 : 2;  // A_hi, B_hi, (A_lo, B_lo)
    static constexpr int T = 2 * WT;            // block tile edge
    static constexpr int MT = WT / 32;          // MFMA tiles per wave edge
    static constexpr int BLK = T / 32 * 2;      // 1 KB fragment blocks per array per chunk
};

// buf: one LDS buffer, [narr][blk_n][64] uint4 flattened; the counts are
// compile-time constants at every (inlined) call.  Row blocks past the padded
// operand (a ragged last tile) load its last block; their outputs are never
// stored.
__device__ __forceinline__ void gram_issue(uint4 *buf, int narr, int blk_n, const uint4 *__restrict__ hi,
                                           const uint4 *__restrict__ lo, int64_t I0, int64_t J0, int64_t rbmax,
                                           int64_t KB, int64_t kb0, int wave, int lane) {
#pragma unroll
    for (int t = 0; t < narr * blk_n / 4; ++t) {
        const int gb = wave + 4 * t;  // 0 .. narr * blk_n - 1
        const int arr = gb / blk_n, blk = gb % blk_n, mb = blk >> 1, ks = blk & 1;
        const uint4 *src = (arr & 2) ? lo : hi;
        int64_t rb = (((arr & 1) ? J0 : I0) >> 5) + mb;
        rb = rb < rbmax ? rb : rbmax;
        __builtin_amdgcn_global_load_lds(src + (rb * KB + kb0 + ks) * 64 + lane, buf + (arr * blk_n + blk) * 64,
                                         16, 0, 0);
    }
}

template <int MAP, bool SPLIT, bool STATS, int WT>
__global__ __launch_bounds__(kGramThreads) void edm_gram_kernel(MapGeom g, const uint16_t *__restrict__ hi,
                                                               const uint16_t *__restrict__ lo,
                                                               const float *__restrict__ norms,
                                                               int64_t n, int64_t dpad,
                                                               float *__restrict__ D,
                                                               unsigned long long *slots) {
    using C = GramCfg<SPLIT, WT>;
    constexpr int T = C::T, MT = C::MT, NP = SPLIT ? 2 : 1;
    uint64_t lin;
    int TX, TY;
    if (!tile2_of<MAP, true>(g, lin, TX, TY)) return;
    constexpr int BUF = C::NARR * C::BLK * 64;  // uint4 per LDS buffer
    __shared__ __attribute__((aligned(16))) uint4 Lb[2 * BUF];
    __shared__ float nA[T], nB[T];

    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    const int64_t I0 = int64_t(TX) * T, J0 = int64_t(TY) * T;
    const bool diag = TX == TY;

    for (int x = t; x < 2 * T; x += kGramThreads) {
        const int64_t r = (x < T ? I0 : J0) + (x & (T - 1));
        (x < T ? nA : nB)[x & (T - 1)] = r < n ? norms[r] : 0.f;
    }

    f32x16_t acc[MT][MT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int c = 0; c < MT; ++c)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[m][c][e] = 0.f;

    const int nst = int(dpad / kGramK);
    const int64_t KB = dpad / 16, rbmax = gram_rows(n) / 32 - 1;
    const uint4 *hi4 = reinterpret_cast<const uint4 *>(hi), *lo4 = reinterpret_cast<const uint4 *>(lo);
    gram_issue(Lb, C::NARR, C::BLK, hi4, lo4, I0, J0, rbmax, KB, 0, w, lane);
    for (int s = 0; s < nst; ++s) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of chunk s have landed
        __syncthreads();                // ... and every wave's; chunk s - 1 is consumed
        const uint4 *cur = Lb + (s & 1) * BUF;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8_t a[NP][MT], b[NP][MT];  // [hi, lo][sub-tile]
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    a[p][m] = __builtin_bit_cast(bf16x8_t, cur[((2 * p) * C::BLK + (wm * MT + m) * 2 + ks) * 64 + lane]);
                    b[p][m] = __builtin_bit_cast(bf16x8_t,
                                                 cur[((2 * p + 1) * C::BLK + (wn * MT + m) * 2 + ks) * 64 + lane]);
                }
            if (ks == 0 && s + 1 < nst)
                gram_issue(Lb + ((s + 1) & 1) * BUF, C::NARR, C::BLK, hi4, lo4, I0, J0, rbmax, KB,
                           int64_t(s + 1) * (kGramK / 16), w, lane);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int c = 0; c < MT; ++c) {
                    acc[m][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][m], b[0][c], acc[m][c], 0, 0, 0);
                    if (SPLIT) {
                        acc[m][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][m], b[NP - 1][c], acc[m][c],
                                                                            0, 0, 0);
                        acc[m][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[NP - 1][m], b[0][c], acc[m][c],
                                                                            0, 0, 0);
                    }
                }
        }
    }

    // 32 x 32 accumulator layout: lane l, element e holds row
    // (e & 3) + 4 (l >> 5) + 8 (e >> 2) and column l & 31 of the MFMA tile.
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int il = wm * WT + m * 32 + (e & 3) + 4 * (lane >> 5) + 8 * (e >> 2);
            const int64_t i = I0 + il;
            if (i >= n) continue;
            const int64_t rowbase = i * n - (i * (i - 1)) / 2 - i;
#pragma unroll
            for (int c = 0; c < MT; ++c) {
                const int jl = wn * WT + c * 32 + (lane & 31);
                const int64_t j = J0 + jl;
                if (j < n && (!diag || j >= i)) {
                    float v = __builtin_fmaf(-2.f, acc[m][c][e], nA[il] + nB[jl]);
                    v = (i == j) ? 0.f : fmaxf(v, 0.f);
                    __builtin_nontemporal_store(v, D + rowbase + j);
                }
            }
        }
    if (STATS) {
        __shared__ unsigned long long red[2][kGramThreads / kWave];
        unsigned long long cnt, cs;
        tile_pairs_le_stats<kGramThreads>(I0, J0, T, T, n, cnt, cs);
        const unsigned long long c = block_sum<unsigned long long, kGramThreads>(cnt, red[0]);
        const unsigned long long h = block_sum<unsigned long long, kGramThreads>(cs, red[1]);
        if (t == 0) stats_add(slots, lin, c, h);
    }
}

template <int MAP, bool SPLIT, int WT>
static void go_gram(const MapGeom &g, const uint16_t *hi, const uint16_t *lo, const float *norms,
                    int64_t n, int64_t dpad, float *D, unsigned long long *slots, hipStream_t s) {
    const dim3 grid = MAP == MAP_BBOX ? dim3(g.nb, g.nb, 1) : grid_for(g.G, kGramThreads);
    if (slots)
        hipLaunchKernelGGL((edm_gram_kernel<MAP, SPLIT, true, WT>), grid, dim3(kGramThreads), 0, s, g, hi, lo,
                           norms, n, dpad, D, slots);
    else
        hipLaunchKernelGGL((edm_gram_kernel<MAP, SPLIT, false, WT>), grid, dim3(kGramThreads), 0, s, g, hi, lo,
                           norms, n, dpad, D, slots);
}

int launch_edm_gram(const MapGeom &g, int tile, const uint16_t *hi, const uint16_t *lo, const float *norms,
                    int64_t n, int64_t dpad, bool split, float *D, unsigned long long *slots,
                    hipStream_t s) {
    prof_begin(K_EDM_GRAM, s);
    map_switch(int(g.map), [&](auto M) {
        constexpr int MAPK = decltype(M)::value;
        if (tile == 256) {
            if (split) go_gram<MAPK, true, 128>(g, hi, lo, norms, n, dpad, D, slots, s);
            else go_gram<MAPK, false, 128>(g, hi, lo, norms, n, dpad, D, slots, s);
        } else {
            if (split) go_gram<MAPK, true, 64>(g, hi, lo, norms, n, dpad, D, slots, s);
            else go_gram<MAPK, false, 64>(g, hi, lo, norms, n, dpad, D, slots, s);
        }
    });
    prof_end(K_EDM_GRAM, s);
    return check_launch("edm_packed (gram)");
}

}  // namespace smx
