// Packed Euclidean distance matrix, FP32 difference form (paper Sec. I and
// II: the EDM is a 2-simplex problem; only the upper triangle is computed and
// stored).
//
// One block of 256 threads owns a T x T tile (X, Y), X <= Y, of the packed
// upper triangle, T = 16 MT (MT = 4 or 8).  The map (lambda2, bounding box or
// linear) only decides which tile a block gets; the body is the same, so
// results are bit-identical across maps.  Per block:
//   * the two T x d row panels of X are staged through LDS in K chunks of 32
//     (row-major, row stride 36 floats: the 16 distinct rows a wave reads with
//     ds_read_b128 land in 16 distinct 16-byte bank groups);
//   * thread (tx, ty) accumulates rows ty + 16 r and columns tx + 16 c
//     (r, c < MT) with one subtract and one FMA per element and dimension --
//     the difference form costs 2 VALU operations per element-dimension, and
//     each ds_read_b128 feeds 4 MT such operations;
//   * stores go to p(i, j) = i n - i (i - 1) / 2 + (j - i): for fixed (r, c) the
//     16 lanes of a row write 16 consecutive floats.
#include "smx_device.h"
#include "smx_internal.h"

namespace smx {

constexpr int kEdmThreads = 256;
constexpr int kEdmKc = 32;
constexpr int kEdmLd = kEdmKc + 4;

// Stage rows [r0, r0 + 16 MT) x dims [k0, k0 + 32) of X into LDS (zero outside):
// slot (row, q) = 8 floats, 4 slots per row, MT / 4 ... MT / 2 slots per thread.
template <int MT, bool VEC>
__device__ __forceinline__ void edm_stage(float *__restrict__ sm, const float *__restrict__ X,
                                          int64_t n, int64_t d, int64_t ldx, int64_t r0, int64_t k0) {
    constexpr int T = 16 * MT;
#pragma unroll
    for (int h = 0; h < T * 4 / kEdmThreads; ++h) {
        const int slot = threadIdx.x + h * kEdmThreads;
        const int row = slot >> 2, q = slot & 3;
        const int64_t gr = r0 + row;
        float v[8];
        if (VEC) {
            // ldx % 4 == 0, 16-byte aligned base, d % 32 == 0: whole chunk in range per row
            if (gr < n) {
                const float4 *src = reinterpret_cast<const float4 *>(X + gr * ldx + k0 + 8 * q);
                const float4 a = src[0], b = src[1];
                v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
                v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) v[e] = 0.f;
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t k = k0 + 8 * q + e;
                v[e] = (gr < n && k < d) ? X[gr * ldx + k] : 0.f;
            }
        }
        float4 *dst = reinterpret_cast<float4 *>(sm + row * kEdmLd + 8 * q);
        dst[0] = make_float4(v[0], v[1], v[2], v[3]);
        dst[1] = make_float4(v[4], v[5], v[6], v[7]);
    }
}

// TILED: the tile-contiguous layout (tile (X, Y) at rank Y(Y+1)/2 + X times T^2,
// element (i, j) at (i mod T) T + (j mod T), entries outside i <= j < n zero).
template <int MAP, int MT, bool VEC, bool STATS, bool TILED>
__global__ __launch_bounds__(kEdmThreads, 3) void edm_diff_kernel(MapGeom g, const float *__restrict__ X,
                                                               int64_t n, int64_t d, int64_t ldx,
                                                               float *__restrict__ D,
                                                               unsigned long long *slots) {
    constexpr int T = 16 * MT;
    uint64_t lin;
    int TX, TY;
    if (!tile2_of<MAP, true>(g, lin, TX, TY)) return;

    __shared__ __attribute__((aligned(16))) float As[T * kEdmLd];
    __shared__ __attribute__((aligned(16))) float Bs[T * kEdmLd];

    const int t = threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    const int64_t r0 = int64_t(TX) * T, c0 = int64_t(TY) * T;
    const bool diag = TX == TY;

    float acc[MT][MT];
#pragma unroll
    for (int r = 0; r < MT; ++r)
#pragma unroll
        for (int c = 0; c < MT; ++c) acc[r][c] = 0.f;

    for (int64_t k0 = 0; k0 < d; k0 += kEdmKc) {
        edm_stage<MT, VEC>(As, X, n, d, ldx, r0, k0);
        if (!diag) edm_stage<MT, VEC>(Bs, X, n, d, ldx, c0, k0);
        __syncthreads();
        const float *Bp = diag ? As : Bs;
#pragma unroll
        for (int kk = 0; kk < kEdmKc; kk += 4) {
            float4 a[MT], b[MT];
#pragma unroll
            for (int r = 0; r < MT; ++r) a[r] = *reinterpret_cast<const float4 *>(As + (ty + 16 * r) * kEdmLd + kk);
#pragma unroll
            for (int c = 0; c < MT; ++c) b[c] = *reinterpret_cast<const float4 *>(Bp + (tx + 16 * c) * kEdmLd + kk);
#pragma unroll
            for (int r = 0; r < MT; ++r)
#pragma unroll
                for (int c = 0; c < MT; ++c) {
                    float u;
                    u = a[r].x - b[c].x; acc[r][c] = __builtin_fmaf(u, u, acc[r][c]);
                    u = a[r].y - b[c].y; acc[r][c] = __builtin_fmaf(u, u, acc[r][c]);
                    u = a[r].z - b[c].z; acc[r][c] = __builtin_fmaf(u, u, acc[r][c]);
                    u = a[r].w - b[c].w; acc[r][c] = __builtin_fmaf(u, u, acc[r][c]);
                }
        }
        __syncthreads();
    }

    // a tile off the diagonal and inside n (nearly every block) stores unmasked
    const bool interior = !diag && r0 + T <= n && c0 + T <= n;
    if (TILED) {
        const uint64_t rank = uint64_t(TY) * (uint64_t(TY) + 1) / 2 + uint64_t(TX);
        float *tileD = D + rank * uint64_t(T * T) + tx;
#pragma unroll
        for (int r = 0; r < MT; ++r) {
            const int64_t i = r0 + ty + 16 * r;
            float *row = tileD + (ty + 16 * r) * T;
#pragma unroll
            for (int c = 0; c < MT; ++c) {
                const int64_t j = c0 + tx + 16 * c;
                row[16 * c] = (interior || (i < n && j < n && j >= i)) ? acc[r][c] : 0.f;
            }
        }
    } else {
#pragma unroll
    for (int r = 0; r < MT; ++r) {
        const int64_t i = r0 + ty + 16 * r;
        if (!interior && i >= n) continue;
        float *row = D + (i * n - (i * (i - 1)) / 2 - i) + c0 + tx;  // p(i, j) = i n - i(i-1)/2 + (j - i)
#pragma unroll
        for (int c = 0; c < MT; ++c) {
            const int64_t j = c0 + tx + 16 * c;
            // plain stores: measured faster than non-temporal ones here
            if (interior ? smx_check(i < n && j < n && j >= i, kCheckStore) : (j < n && (!diag || j >= i)))
                row[16 * c] = acc[r][c];
        }
    }
    }
    if (STATS) {
        __shared__ unsigned long long red[2][kEdmThreads / kWave];
        unsigned long long cnt, cs;
        tile_pairs_le_stats<kEdmThreads>(r0, c0, T, T, n, cnt, cs);
        const unsigned long long c = block_sum<unsigned long long, kEdmThreads>(cnt, red[0]);
        const unsigned long long h = block_sum<unsigned long long, kEdmThreads>(cs, red[1]);
        if (t == 0) stats_add(slots, lin, c, h);
    }
}

template <int MAP, int MT, bool VEC, bool TILED>
static void go_edm(const MapGeom &g, const float *X, int64_t n, int64_t d, int64_t ldx, float *D,
                   unsigned long long *slots, hipStream_t s) {
    const dim3 grid = MAP == MAP_BBOX ? dim3(g.nb, g.nb, 1) : grid_for(g.G, kEdmThreads);
    if (slots)
        hipLaunchKernelGGL((edm_diff_kernel<MAP, MT, VEC, true, TILED>), grid, dim3(kEdmThreads), 0, s, g, X, n,
                           d, ldx, D, slots);
    else
        hipLaunchKernelGGL((edm_diff_kernel<MAP, MT, VEC, false, TILED>), grid, dim3(kEdmThreads), 0, s, g, X, n,
                           d, ldx, D, slots);
}

template <int MAP>
static void go_edm_map(const MapGeom &g, int tile, bool vec, bool tiled, const float *X, int64_t n, int64_t d,
                       int64_t ldx, float *D, unsigned long long *slots, hipStream_t s) {
    if (tiled) {  // the tile-contiguous layout uses 128-wide tiles at every n
        if (vec) go_edm<MAP, 8, true, true>(g, X, n, d, ldx, D, slots, s);
        else go_edm<MAP, 8, false, true>(g, X, n, d, ldx, D, slots, s);
    } else if (tile == 128) {
        if (vec) go_edm<MAP, 8, true, false>(g, X, n, d, ldx, D, slots, s);
        else go_edm<MAP, 8, false, false>(g, X, n, d, ldx, D, slots, s);
    } else {
        if (vec) go_edm<MAP, 4, true, false>(g, X, n, d, ldx, D, slots, s);
        else go_edm<MAP, 4, false, false>(g, X, n, d, ldx, D, slots, s);
    }
}

int launch_edm_diff(const MapGeom &g, int tile, const float *X, int64_t n, int64_t d, int64_t ldx, float *D,
                    unsigned long long *slots, bool tiled, hipStream_t s) {
    const bool vec = (ldx % 4 == 0) && (d % kEdmKc == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
    prof_begin(K_EDM_DIFF, s);
    for_each_launch(g, [&](auto M, const MapGeom &gg) {
        go_edm_map<decltype(M)::value>(gg, tile, vec, tiled, X, n, d, ldx, D, slots, s);
    });
    prof_end(K_EDM_DIFF, s);
    return check_launch("edm_packed (fp32 diff)");
}

SMX_CHECK_READER(check_flags_edm)

}  // namespace smx
