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
// triangle, each wave 64 x 64 in MFMA tiles of 32 x 32.  K advances in steps
// of 16 BF16 through a 32 KB ring of LDS slots filled directly from global
// memory in MFMA fragment order (see the staging notes below), so the loads
// of the next steps are in flight while the matrix cores run the current one.
#include "smx_device.h"
#include "smx_internal.h"

namespace smx {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

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
// later reads back as its operand (rows mb*32 + (s & 31), k = 8*(s >> 5) .. +7
// of one 16-wide k step), so an operand read is base + 16*lane (no bank
// conflicts) and staging costs no VGPRs.
//
// Pipeline.  One stage = one 16-wide k step of both panels.  A ring of S
// stages keeps S - 1 steps of loads in flight: at step s a wave waits until
// only the loads of steps s+1 .. s+S-2 are outstanding (loads complete in
// issue order), the block synchronises, the loads of step s+S-1 go into the
// slot step s-1 used, and the MFMAs of step s run.
//
// WT = wave tile: the block tile is T = 2 WT, each wave owns WT / 32 x WT / 32
// MFMA tiles.  T = 128 (WT = 64) with a 32 KB ring (4 slots of 8 KB plain, 2
// of 16 KB split): at most 128 registers per lane and 33 KB of LDS, so four
// blocks share a CU and the store-heavy epilogue of one overlaps the others'
// k loops.  Measured on MI355X against 2 blocks per CU with 64 KB rings and
// against wider slots (2 or 4 k steps each, 32-64 KB): those were 4-20%
// slower; so were persistent grids that overlap each tile's stores with the
// next tile's k loop inside one block.
template <bool SPLIT, int WT>
struct GramCfg {
    static constexpr int NARR = SPLIT ? 4 : 2;     // A_hi, B_hi, (A_lo, B_lo)
    static constexpr int T = 2 * WT;               // block tile edge
    static constexpr int MT = WT / 32;             // MFMA tiles per wave edge
    static constexpr int RB = T / 32;              // 32-row blocks per panel
    static constexpr int KS = 1;                   // 16-wide k blocks per stage
    static constexpr int STAGE = NARR * RB * KS;   // 1 KB blocks per stage
    static constexpr int LPW = STAGE / 4;          // loads per wave per stage
    static constexpr int S = SPLIT ? 2 : 4;         // ring depth: 32 KB either way
};

// One 16-byte store of four packed distances, ordinary or marked non-temporal.
// The distances are written once and never read back by the kernel; streaming
// them past the caches keeps the L2 for the operand panels, which pays once the
// k loop is long.  Measured on MI355X at n = 32768 (ms, ordinary / streaming):
// plain d = 32 0.58 / 0.77, d = 128 0.64 / 0.76, d = 256 0.77 / 0.76, d = 512
// 1.02 / 0.80; split d = 64 0.67 / 0.79, d = 128 0.81 / 0.80, d = 512 1.71 /
// 1.69.  The streaming stores hold about 2.8 TB/s whatever d; the ordinary
// ones reach 3.7 TB/s alone but slow the k loop down as d grows.  The
// tile-contiguous layout (aligned 64 KB runs) follows the same rule: plain
// d = 32 0.37 / 0.37, d = 512 0.83 / 0.74.  (A HIP float4 assignment here
// compiled to a 12-byte and a 4-byte store, hence the vector type.)
template <bool NT>
__device__ __forceinline__ void store4(float *p, float4 v) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 w = {v.x, v.y, v.z, v.w};
    if constexpr (NT)
        __builtin_nontemporal_store(w, reinterpret_cast<f4 *>(p));
    else
        *reinterpret_cast<f4 *>(p) = w;
}

// One stage's loads into buf ([narr][rb_n][64] uint4); the counts are
// compile-time constants at every (inlined) call.  Row blocks past the padded
// operand (a ragged last tile) load its last block; their outputs are never
// stored.
__device__ __forceinline__ void gram_issue(uint4 *buf, int narr, int rb_n, int ks, const uint4 *__restrict__ hi,
                                           const uint4 *__restrict__ lo, int64_t I0, int64_t J0, int64_t rbmax,
                                           int64_t KB, int64_t kb, int wave, int lane) {
#pragma unroll
    for (int t = 0; t < narr * rb_n * ks / 4; ++t) {
        const int gb = wave + 4 * t;  // 0 .. narr * rb_n * ks - 1: [array][row block][k block]
        const int arr = gb / (rb_n * ks), rem = gb % (rb_n * ks), mb = rem / ks, kk = rem % ks;
        const uint4 *src = (arr & 2) ? lo : hi;
        int64_t rb = (((arr & 1) ? J0 : I0) >> 5) + mb;
        rb = rb < rbmax ? rb : rbmax;
        __builtin_amdgcn_global_load_lds(src + (rb * KB + kb + kk) * 64 + lane, buf + gb * 64, 16, 0, 0);
    }
}

// s_waitcnt with vmcnt <= N (N < 64) and no wait on the other counters.
template <int N>
__device__ __forceinline__ void wait_vm() {
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
template <int LPW, int A>
__device__ __forceinline__ void wait_vm_ahead(int ahead) {
    if constexpr (A < 0) {
        return;
    } else {
        if (ahead == A) wait_vm<A * LPW>();
        else wait_vm_ahead<LPW, A - 1>(ahead);
    }
}

// Operand fragments are read from the ring with ds_read_b128 written out as
// inline assembly: the compiler does not model the LDS writes of the
// global-to-LDS loads, so it would either wait for every load in flight
// before each LDS read or treat the ring as never written.  The reads are
// waited for explicitly (lds_wait), and that wait names the fragment
// registers so no use can move above it.
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return static_cast<uint32_t>(reinterpret_cast<uintptr_t>(p));
}
__device__ __forceinline__ bf16x8_t lds_frag(uint32_t addr) {
    bf16x8_t v;
    asm volatile("ds_read_b128 %0, %1" : "=v"(v) : "v"(addr) : "memory");
    return v;
}
template <int NP, int MT>
__device__ __forceinline__ void lds_wait(bf16x8_t (&a)[NP][MT], bf16x8_t (&b)[NP][MT]) {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int m = 0; m < MT; ++m) asm volatile("" : "+v"(a[p][m]), "+v"(b[p][m]));
}

// TILED: the tile-contiguous layout (tile (X, Y) at rank Y(Y+1)/2 + X times T^2,
// element (i, j) at (i mod T) T + (j mod T), entries outside i <= j < n zero).
// NT: the output stores are streaming (non-temporal); chosen at compile time,
// since the compiler merges the two arms of a run-time choice into one ordinary
// store.
template <int MAP, bool SPLIT, bool STATS, int WT, bool TILED, bool NT>
__global__ __launch_bounds__(kGramThreads, 4) void edm_gram_kernel(MapGeom g, const uint16_t *__restrict__ hi,
                                                               const uint16_t *__restrict__ lo,
                                                               const float *__restrict__ norms,
                                                               int64_t n, int64_t dpad,
                                                               float *__restrict__ D,
                                                               unsigned long long *slots) {
    using C = GramCfg<SPLIT, WT>;
    constexpr int T = C::T, MT = C::MT, NP = SPLIT ? 2 : 1, S = C::S;
    constexpr int BUF = C::STAGE * 64;  // uint4 per ring slot
    static_assert(S * BUF * 16 >= 2 * 32 * T * 4, "the epilogue stages 64 tile rows in the ring");
    uint64_t lin;
    int TX, TY;
    if (MAP == MAP_LAMBDA) {
        // Each XCD takes one contiguous range of Pi2, walked in patches (w_x by
        // w_y ids: 8 x 16 plain, 16 x 8 split) so that its L2 keeps the row and
        // column panels of the tiles it runs at once: operands fetched from
        // beyond L2 4.2 -> 0.8 GB plain, 8.6 -> 2.8 GB split.  Column-major order
        // (w_y fastest, whose concurrent tiles extend the same packed rows) is
        // the faster one for the stores alone, but with the non-temporal stores
        // the patches took 5-10% less time at d = 512.
        lin = launch_index();
        if (lin >= g.G) return;
        const uint32_t id = xcd_remap(uint32_t(lin), uint32_t(g.G));
        if (!lambda2(SPLIT ? lambda2_patch_to_xfast(id, g.lg, 4, 3) : lambda2_patch_to_xfast(id, g.lg, 3, 4), g.lg,
                     g.nb, TX, TY))
            return;
        if (SMX_CHECKED && !smx_check(0 <= TX && TX <= TY && TY < g.nb, kCheckMap)) return;
    } else if (!tile2_of<MAP, true>(g, lin, TX, TY)) {
        return;
    }
    __shared__ __attribute__((aligned(16))) uint4 Lb[S * BUF];
    __shared__ __attribute__((aligned(16))) float nA[T], nB[T];

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

    constexpr int KS = C::KS;
    const int nst = int(dpad / (16 * KS));  // stages of KS 16-wide k blocks
    const int64_t KB = dpad / 16, rbmax = gram_rows(n) / 32 - 1;
    const uint4 *hi4 = reinterpret_cast<const uint4 *>(hi), *lo4 = reinterpret_cast<const uint4 *>(lo);
    for (int p = 0; p < S - 1 && p < nst; ++p)
        gram_issue(Lb + p * BUF, C::NARR, C::RB, KS, hi4, lo4, I0, J0, rbmax, KB, int64_t(p) * KS, w, lane);
    const uint32_t ring = lds_addr(Lb);
    bf16x8_t a[2][NP][MT], b[2][NP][MT];  // [k block parity][hi, lo][sub-tile]
    for (int st = 0; st < nst; ++st) {
        const int ahead = nst - 1 - st < S - 2 ? nst - 1 - st : S - 2;
        wait_vm_ahead<C::LPW, S - 2>(ahead);  // this wave's loads of stage st have landed
        __builtin_amdgcn_s_barrier();           // ... and every wave's; stage st - 1 is consumed
        if (st + S - 1 < nst)
            gram_issue(Lb + ((st + S - 1) % S) * BUF, C::NARR, C::RB, KS, hi4, lo4, I0, J0, rbmax, KB,
                       int64_t(st + S - 1) * KS, w, lane);
        const uint32_t cur = ring + uint32_t((st % S) * BUF) * 16u + uint32_t(lane) * 16u;
        // k blocks of the stage, the fragments of block kk + 1 read while block kk multiplies
        auto rd = [&](int kk, bf16x8_t(&fa)[NP][MT], bf16x8_t(&fb)[NP][MT]) {
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    fa[p][m] = lds_frag(cur + uint32_t((((2 * p) * C::RB + wm * MT + m) * KS + kk) * 64 * 16));
                    fb[p][m] = lds_frag(cur + uint32_t((((2 * p + 1) * C::RB + wn * MT + m) * KS + kk) * 64 * 16));
                }
        };
        rd(0, a[0], b[0]);
        lds_wait<NP, MT>(a[0], b[0]);
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const int q = kk & 1;
            if (kk + 1 < KS) rd(kk + 1, a[q ^ 1], b[q ^ 1]);
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int c = 0; c < MT; ++c) {
                    acc[m][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[q][0][m], b[q][0][c], acc[m][c], 0, 0, 0);
                    if (SPLIT) {
                        acc[m][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[q][0][m], b[q][NP - 1][c], acc[m][c], 0,
                                                                            0, 0);
                        acc[m][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[q][NP - 1][m], b[q][0][c], acc[m][c], 0,
                                                                            0, 0);
                    }
                }
            if (kk + 1 < KS) lds_wait<NP, MT>(a[q ^ 1], b[q ^ 1]);
        }
    }

    // Epilogue.  32 x 32 accumulator layout: lane l, element e holds row
    // (e & 3) + 4 (l >> 5) + 8 (e >> 2) and column l & 31 of the MFMA tile.
    // Per pass m the four waves stage 64 whole rows of the tile (32 from each
    // row half) in the (now idle) ring; then each wave writes 16 of them, two
    // 512-byte tile rows per store instruction, so that only the two ends of a
    // tile row share a 128-byte line with the neighbouring tiles (half-row
    // pieces per wave: 0.995 against 0.938 ms plain, 1.855 against 1.829 split).
    // Tiles off the diagonal and inside n (all but a thin fringe) store
    // unmasked.
    static_assert(T == 128 && kGramThreads == 256, "the store loop assumes 4 waves and 128-wide tile rows");
    float *St = reinterpret_cast<float *>(Lb);  // [2 * 32 rows][T], the rows of one pass
    const bool interior = !diag && I0 + T <= n && J0 + T <= n;
    float nb[MT];
#pragma unroll
    for (int c = 0; c < MT; ++c) nb[c] = nB[wn * WT + c * 32 + (lane & 31)];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        __syncthreads();  // the ring (k loop) or the previous pass's rows are consumed
        float na[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 r4 = *reinterpret_cast<const float4 *>(&nA[wm * WT + m * 32 + 8 * q + 4 * (lane >> 5)]);
            na[4 * q + 0] = r4.x; na[4 * q + 1] = r4.y; na[4 * q + 2] = r4.z; na[4 * q + 3] = r4.w;
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int rl = (e & 3) + 4 * (lane >> 5) + 8 * (e >> 2);
#pragma unroll
            for (int c = 0; c < MT; ++c) {
                float v = fmaxf(__builtin_fmaf(-2.f, acc[m][c][e], na[e] + nb[c]), 0.f);
                // on a diagonal tile, element (il, il) is the diagonal: exactly 0
                v = (diag && wm * WT + m * 32 + rl == wn * WT + c * 32 + (lane & 31)) ? 0.f : v;
                St[(wm * 32 + rl) * T + wn * WT + c * 32 + (lane & 31)] = v;
            }
        }
        __syncthreads();
        // each wave writes 16 whole tile rows, two per instruction
#pragma unroll
        for (int it = 0; it < 8; ++it) {
            const int r = w * 16 + 2 * it + (lane >> 5), cl = 4 * (lane & 31);
            const int64_t i = I0 + (r >> 5) * WT + m * 32 + (r & 31), j = J0 + cl;
            const float4 v = *reinterpret_cast<const float4 *>(St + r * T + cl);
            if (TILED) {
                const uint64_t rank = uint64_t(TY) * (uint64_t(TY) + 1) / 2 + uint64_t(TX);
                float *tdst = D + rank * uint64_t(T * T) + uint64_t(i - I0) * T + uint64_t(j - J0);
                float4 o = v;
                if (!interior) {
                    o.x = (i < n && j + 0 < n && j + 0 >= i) ? v.x : 0.f;
                    o.y = (i < n && j + 1 < n && j + 1 >= i) ? v.y : 0.f;
                    o.z = (i < n && j + 2 < n && j + 2 >= i) ? v.z : 0.f;
                    o.w = (i < n && j + 3 < n && j + 3 >= i) ? v.w : 0.f;
                }
                store4<NT>(tdst, o);  // 16-byte aligned: tiles start at multiples of T^2
                continue;
            }
            float *dst = D + (i * n - (i * (i - 1)) / 2 - i) + j;
            if (interior) {
                if (smx_check(i < n && j >= i && j + 3 < n, kCheckStore))
                    store4<NT>(dst, v);  // 4-byte aligned: the packed rows start anywhere
            } else if (i < n) {
                const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (j + q < n && j + q >= i) dst[q] = vv[q];
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


template <int MAP, bool SPLIT, int WT, bool TILED, bool NT>
static void go_gram(const MapGeom &g, const uint16_t *hi, const uint16_t *lo, const float *norms,
                    int64_t n, int64_t dpad, float *D, unsigned long long *slots, hipStream_t s) {
    const dim3 grid = MAP == MAP_BBOX ? dim3(g.nb, g.nb, 1) : grid_for(g.G, kGramThreads);
    if (slots)
        hipLaunchKernelGGL((edm_gram_kernel<MAP, SPLIT, true, WT, TILED, NT>), grid, dim3(kGramThreads), 0, s, g,
                           hi, lo, norms, n, dpad, D, slots);
    else
        hipLaunchKernelGGL((edm_gram_kernel<MAP, SPLIT, false, WT, TILED, NT>), grid, dim3(kGramThreads), 0, s, g,
                           hi, lo, norms, n, dpad, D, slots);
}

// Streaming stores once the k loop is long enough for the operand panels' L2
// residency to matter more than the stores' own rate (see store4).
static bool gram_streaming(int64_t dpad, bool split) { return (split ? 2 : 1) * dpad >= 256; }

int launch_edm_gram(const MapGeom &g, int tile, const uint16_t *hi, const uint16_t *lo, const float *norms,
                    int64_t n, int64_t dpad, bool split, float *D, unsigned long long *slots, bool tiled,
                    hipStream_t s) {
    prof_begin(K_EDM_GRAM, s);
    for_each_launch(g, [&](auto M, const MapGeom &gg) {
        constexpr int MAPK = decltype(M)::value;
        constexpr int WT = kGramTile / 2;
        (void)tile;  // kGramTile
        const bool nt = gram_streaming(dpad, split);
        if (tiled && nt) {
            if (split) go_gram<MAPK, true, WT, true, true>(gg, hi, lo, norms, n, dpad, D, slots, s);
            else go_gram<MAPK, false, WT, true, true>(gg, hi, lo, norms, n, dpad, D, slots, s);
        } else if (tiled) {
            if (split) go_gram<MAPK, true, WT, true, false>(gg, hi, lo, norms, n, dpad, D, slots, s);
            else go_gram<MAPK, false, WT, true, false>(gg, hi, lo, norms, n, dpad, D, slots, s);
        } else if (nt) {
            if (split) go_gram<MAPK, true, WT, false, true>(gg, hi, lo, norms, n, dpad, D, slots, s);
            else go_gram<MAPK, false, WT, false, true>(gg, hi, lo, norms, n, dpad, D, slots, s);
        } else {
            if (split) go_gram<MAPK, true, WT, false, false>(gg, hi, lo, norms, n, dpad, D, slots, s);
            else go_gram<MAPK, false, WT, false, false>(gg, hi, lo, norms, n, dpad, D, slots, s);
        }
    });
    prof_end(K_EDM_GRAM, s);
    return check_launch("edm_packed (gram)");
}

SMX_CHECK_READER(check_flags_gram)

}  // namespace smx
