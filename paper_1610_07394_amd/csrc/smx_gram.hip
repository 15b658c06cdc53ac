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
// Block: 256 threads (4 waves as 2 x 2), tile 128 x 128 of the packed upper
// triangle, each wave 64 x 64 = 2 x 2 MFMA tiles of 32 x 32.  K advances in
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

// One wave per row: hi / lo BF16 copies (zero padded to dpad) and the FP32
// squared norm sum_k x_k^2 (lane-strided FMA sums, then a fixed wave tree).
__global__ __launch_bounds__(256) void gram_prep_kernel(const float *__restrict__ X, int64_t n,
                                                        int64_t d, int64_t ldx, int64_t dpad,
                                                        uint16_t *__restrict__ hi,
                                                        uint16_t *__restrict__ lo,
                                                        float *__restrict__ norms) {
    const int lane = threadIdx.x & 63;
    const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    float acc = 0.f;
    for (int64_t k = lane; k < dpad; k += 64) {
        const float x = k < d ? X[row * ldx + k] : 0.f;
        acc = __builtin_fmaf(x, x, acc);
        const uint16_t h = bf16_rne(x);
        hi[row * dpad + k] = h;
        if (lo != nullptr) lo[row * dpad + k] = bf16_rne(x - bf16_to_f32(h));
    }
    acc = wave_sum(acc);
    if (lane == 0) norms[row] = acc;
}

int launch_gram_prep(const float *X, int64_t n, int64_t d, int64_t ldx, int64_t dpad, uint16_t *hi,
                     uint16_t *lo, float *norms, bool split, hipStream_t s) {
    prof_begin(K_GRAM_PREP, s);
    hipLaunchKernelGGL(gram_prep_kernel, dim3(uint32_t((n + 3) / 4)), dim3(256), 0, s, X, n, d, ldx,
                       dpad, hi, split ? lo : nullptr, norms);
    prof_end(K_GRAM_PREP, s);
    return check_launch("gram prep");
}

// Staging.  Every MFMA operand fragment travels from global memory straight
// into LDS with global_load_lds_dwordx4: one wave load fills a 1 KB block,
// lane s writing the 16 bytes it later reads back as its operand.  Block
// (mb, ks) of a 128-row panel chunk holds rows mb*32 + (s & 31), k =
// ks*16 + 8*(s >> 5) .. +7, so an operand read is base + 16*lane (no bank
// conflicts) and staging costs no VGPRs.  Two LDS buffers alternate: a wave
// reads all fragments of chunk s into registers, then issues the loads of
// chunk s + 1 into the other buffer, then runs the MFMAs of chunk s while those
// loads are in flight.
template <bool SPLIT>
struct GramCfg {
    static constexpr int NARR = SPLIT ? 4 : 2;  // A_hi, B_hi, (A_lo, B_lo)
    static constexpr int LPW = NARR * 8 / 4;    // wave loads per chunk per wave
};

typedef uint4 GramBuf[8][64];  // one array's 128 x 32 chunk in fragment order

template <bool SPLIT>
__device__ __forceinline__ void gram_issue(GramBuf *buf, const uint16_t *__restrict__ hi,
                                           const uint16_t *__restrict__ lo, int64_t I0, int64_t J0,
                                           int64_t n, int64_t dpad, int64_t k0, int wave, int lane) {
#pragma unroll
    for (int t = 0; t < GramCfg<SPLIT>::LPW; ++t) {
        const int gb = wave + 4 * t;  // 0 .. 8 NARR - 1
        const int arr = gb >> 3, blk = gb & 7, mb = blk >> 1, ks = blk & 1;
        const uint16_t *src = (arr & 2) ? lo : hi;
        int64_t row = ((arr & 1) ? J0 : I0) + mb * 32 + (lane & 31);
        row = row < n ? row : n - 1;  // rows past n load row n-1; their outputs are never stored
        const uint16_t *g = src + row * dpad + k0 + ks * 16 + 8 * (lane >> 5);
        __builtin_amdgcn_global_load_lds(g, &buf[arr][blk][0], 16, 0, 0);
    }
}

template <int MAP, bool SPLIT, bool STATS>
__global__ __launch_bounds__(kGramThreads) void edm_gram_kernel(MapGeom g, const uint16_t *__restrict__ hi,
                                                               const uint16_t *__restrict__ lo,
                                                               const float *__restrict__ norms,
                                                               int64_t n, int64_t dpad,
                                                               float *__restrict__ D,
                                                               unsigned long long *slots) {
    uint64_t lin;
    int TX, TY;
    if (!tile2_of<MAP, true>(g, lin, TX, TY)) return;
    constexpr int NARR = GramCfg<SPLIT>::NARR, NP = SPLIT ? 2 : 1;
    __shared__ __attribute__((aligned(16))) GramBuf Lb[2][NARR];
    __shared__ float nA[kGramTile], nB[kGramTile];

    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
    const int64_t I0 = int64_t(TX) * kGramTile, J0 = int64_t(TY) * kGramTile;
    const bool diag = TX == TY;

    if (t < kGramTile) nA[t] = I0 + t < n ? norms[I0 + t] : 0.f;
    else nB[t - kGramTile] = J0 + t - kGramTile < n ? norms[J0 + t - kGramTile] : 0.f;

    f32x16_t acc[2][2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[m][c][e] = 0.f;

    const int nst = int(dpad / kGramK);
    gram_issue<SPLIT>(Lb[0], hi, lo, I0, J0, n, dpad, 0, w, lane);
    for (int s = 0; s < nst; ++s) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of chunk s have landed
        __syncthreads();                // ... and every wave's; chunk s - 1 is consumed
        const GramBuf *cur = Lb[s & 1];
        bf16x8_t a[2][NP][2], b[2][NP][2];  // [k-step][hi, lo][sub-tile]
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    a[ks][p][m] = __builtin_bit_cast(bf16x8_t, cur[2 * p][(wm * 2 + m) * 2 + ks][lane]);
                    b[ks][p][m] = __builtin_bit_cast(bf16x8_t, cur[2 * p + 1][(wn * 2 + m) * 2 + ks][lane]);
                }
        if (s + 1 < nst)
            gram_issue<SPLIT>(Lb[(s + 1) & 1], hi, lo, I0, J0, n, dpad, int64_t(s + 1) * kGramK, w, lane);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    acc[m][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks][0][m], b[ks][0][c], acc[m][c], 0, 0, 0);
                    if (SPLIT) {
                        acc[m][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks][0][m], b[ks][NP - 1][c], acc[m][c],
                                                                            0, 0, 0);
                        acc[m][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ks][NP - 1][m], b[ks][0][c], acc[m][c],
                                                                            0, 0, 0);
                    }
                }
    }

    // 32 x 32 accumulator layout: lane l, element e holds row
    // (e & 3) + 4 (l >> 5) + 8 (e >> 2) and column l & 31 of the MFMA tile.
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int il = wm * 64 + m * 32 + (e & 3) + 4 * (lane >> 5) + 8 * (e >> 2);
            const int64_t i = I0 + il;
            if (i >= n) continue;
            const int64_t rowbase = i * n - (i * (i - 1)) / 2 - i;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int jl = wn * 64 + c * 32 + (lane & 31);
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
        tile_pairs_le_stats<kGramThreads>(I0, J0, kGramTile, kGramTile, n, cnt, cs);
        const unsigned long long c = block_sum<unsigned long long, kGramThreads>(cnt, red[0]);
        const unsigned long long h = block_sum<unsigned long long, kGramThreads>(cs, red[1]);
        if (t == 0) stats_add(slots, lin, c, h);
    }
}
template <int MAP, bool SPLIT>
static void go_gram(const MapGeom &g, const uint16_t *hi, const uint16_t *lo, const float *norms,
                    int64_t n, int64_t dpad, float *D, unsigned long long *slots, hipStream_t s) {
    const dim3 grid = MAP == MAP_BBOX ? dim3(g.nb, g.nb, 1) : grid_for(g.G, kGramThreads);
    if (slots)
        hipLaunchKernelGGL((edm_gram_kernel<MAP, SPLIT, true>), grid, dim3(kGramThreads), 0, s, g, hi, lo,
                           norms, n, dpad, D, slots);
    else
        hipLaunchKernelGGL((edm_gram_kernel<MAP, SPLIT, false>), grid, dim3(kGramThreads), 0, s, g, hi, lo,
                           norms, n, dpad, D, slots);
}

int launch_edm_gram(const MapGeom &g, const uint16_t *hi, const uint16_t *lo, const float *norms,
                    int64_t n, int64_t dpad, bool split, float *D, unsigned long long *slots,
                    hipStream_t s) {
    prof_begin(K_EDM_GRAM, s);
    map_switch(int(g.map), [&](auto M) {
        constexpr int MAPK = decltype(M)::value;
        if (split) go_gram<MAPK, true>(g, hi, lo, norms, n, dpad, D, slots, s);
        else go_gram<MAPK, false>(g, hi, lo, norms, n, dpad, D, slots, s);
    });
    prof_end(K_EDM_GRAM, s);
    return check_launch("edm_packed (gram)");
}

}  // namespace smx
