// Packed Euclidean distance matrix, FP32 difference form (paper Sec. I and
// II: the EDM is a 2-simplex problem; only the upper triangle is computed and
// stored).
//
// One block of 256 threads owns a 64 x 64 tile (X, Y), X <= Y, of the packed
// upper triangle.  The map (lambda2, bounding box or linear) only decides
// which tile a block gets; the body is the same, so results are bit-identical
// across maps.  Per block:
//   * the two 64 x d row panels of X are staged through LDS in K chunks of 32
//     (row-major, row stride 36 floats: the 16 distinct rows a wave reads with
//     ds_read_b128 land in 16 distinct 16-byte bank groups);
//   * thread (tx, ty) accumulates rows ty + 16 r and columns tx + 16 c
//     (r, c < 4) with one subtract and one FMA per element and dimension --
//     the difference form costs 2 VALU operations per element-dimension;
//   * stores go to p(i, j) = i n - i (i - 1) / 2 + (j - i): for fixed (r, c) the
//     16 lanes of a row write 16 consecutive floats.
#include "smx_device.h"
#include "smx_internal.h"

namespace smx {

constexpr int kEdmThreads = 256;
constexpr int kEdmKc = 32;
constexpr int kEdmLd = kEdmKc + 4;

template <int MAP>
__device__ __forceinline__ bool edm_tile(const MapGeom &g, uint64_t &lin, int &X, int &Y) {
    if (MAP == MAP_BBOX) {
        X = int(blockIdx.x);
        Y = int(blockIdx.y);
        lin = uint64_t(Y) * uint64_t(g.nb) + uint64_t(X);
        return X <= Y;
    }
    lin = launch_index();
    if (lin >= g.G) return false;
    const uint32_t id = xcd_remap(uint32_t(lin), uint32_t(g.G));
    lin = id;
    if (MAP == MAP_LAMBDA) return lambda2(id, g.lg, g.nb, X, Y);
    linear2(id, X, Y);
    return true;
}

// Stage rows [r0, r0 + 64) x dims [k0, k0 + 32) of X into LDS (zero outside).
template <bool VEC>
__device__ __forceinline__ void edm_stage(float *__restrict__ sm, const float *__restrict__ X,
                                          int64_t n, int64_t d, int64_t ldx, int64_t r0, int64_t k0) {
    const int t = threadIdx.x;
    const int row = t >> 2, q = t & 3;  // 64 rows x 4 quarters of 8 floats
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

template <int MAP, bool VEC, bool STATS>
__global__ __launch_bounds__(kEdmThreads) void edm_diff_kernel(MapGeom g, const float *__restrict__ X,
                                                               int64_t n, int64_t d, int64_t ldx,
                                                               float *__restrict__ D,
                                                               unsigned long long *slots) {
    uint64_t lin;
    int TX, TY;
    if (!edm_tile<MAP>(g, lin, TX, TY)) return;

    __shared__ __attribute__((aligned(16))) float As[kEdmTile * kEdmLd];
    __shared__ __attribute__((aligned(16))) float Bs[kEdmTile * kEdmLd];

    const int t = threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    const int64_t r0 = int64_t(TX) * kEdmTile, c0 = int64_t(TY) * kEdmTile;
    const bool diag = TX == TY;

    float acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.f;

    for (int64_t k0 = 0; k0 < d; k0 += kEdmKc) {
        edm_stage<VEC>(As, X, n, d, ldx, r0, k0);
        if (!diag) edm_stage<VEC>(Bs, X, n, d, ldx, c0, k0);
        __syncthreads();
        const float *Bp = diag ? As : Bs;
#pragma unroll
        for (int kk = 0; kk < kEdmKc; kk += 4) {
            float4 a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = *reinterpret_cast<const float4 *>(As + (ty + 16 * r) * kEdmLd + kk);
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = *reinterpret_cast<const float4 *>(Bp + (tx + 16 * c) * kEdmLd + kk);
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    float u;
                    u = a[r].x - b[c].x; acc[r][c] = __builtin_fmaf(u, u, acc[r][c]);
                    u = a[r].y - b[c].y; acc[r][c] = __builtin_fmaf(u, u, acc[r][c]);
                    u = a[r].z - b[c].z; acc[r][c] = __builtin_fmaf(u, u, acc[r][c]);
                    u = a[r].w - b[c].w; acc[r][c] = __builtin_fmaf(u, u, acc[r][c]);
                }
        }
        __syncthreads();
    }

#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = r0 + ty + 16 * r;
        if (i >= n) continue;
        const int64_t rowbase = i * n - (i * (i - 1)) / 2 - i;  // p(i, j) = rowbase + j
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t j = c0 + tx + 16 * c;
            if (j < n && (!diag || j >= i)) __builtin_nontemporal_store(acc[r][c], D + rowbase + j);
        }
    }
    if (STATS) {
        __shared__ unsigned long long red[2][kEdmThreads / kWave];
        unsigned long long cnt, cs;
        tile_pairs_le_stats<kEdmThreads>(r0, c0, kEdmTile, kEdmTile, n, cnt, cs);
        const unsigned long long c = block_sum<unsigned long long, kEdmThreads>(cnt, red[0]);
        const unsigned long long h = block_sum<unsigned long long, kEdmThreads>(cs, red[1]);
        if (t == 0) stats_add(slots, lin, c, h);
    }
}

template <int MAP, bool VEC>
static void go_edm(const MapGeom &g, const float *X, int64_t n, int64_t d, int64_t ldx, float *D,
                   unsigned long long *slots, hipStream_t s) {
    const dim3 grid = MAP == MAP_BBOX ? dim3(g.nb, g.nb, 1) : grid_for(g.G, kEdmThreads);
    if (slots)
        hipLaunchKernelGGL((edm_diff_kernel<MAP, VEC, true>), grid, dim3(kEdmThreads), 0, s, g, X, n, d,
                           ldx, D, slots);
    else
        hipLaunchKernelGGL((edm_diff_kernel<MAP, VEC, false>), grid, dim3(kEdmThreads), 0, s, g, X, n, d,
                           ldx, D, slots);
}

int launch_edm_diff(const MapGeom &g, const float *X, int64_t n, int64_t d, int64_t ldx, float *D,
                    unsigned long long *slots, hipStream_t s) {
    const bool vec = (ldx % 4 == 0) && (d % kEdmKc == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
    prof_begin(K_EDM_DIFF, s);
    const int map = int(g.map);
    if (map == MAP_LAMBDA) {
        if (vec) go_edm<MAP_LAMBDA, true>(g, X, n, d, ldx, D, slots, s);
        else go_edm<MAP_LAMBDA, false>(g, X, n, d, ldx, D, slots, s);
    } else if (map == MAP_BBOX) {
        if (vec) go_edm<MAP_BBOX, true>(g, X, n, d, ldx, D, slots, s);
        else go_edm<MAP_BBOX, false>(g, X, n, d, ldx, D, slots, s);
    } else {
        if (vec) go_edm<MAP_LINEAR, true>(g, X, n, d, ldx, D, slots, s);
        else go_edm<MAP_LINEAR, false>(g, X, n, d, ldx, D, slots, s);
    }
    prof_end(K_EDM_DIFF, s);
    return check_launch("edm_packed (fp32 diff)");
}

}  // namespace smx
