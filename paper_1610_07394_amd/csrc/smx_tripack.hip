// Packed per-triplet Axilrod-Teller energies on the 3-simplex: the tetrahedral
// analogue of the packed EDM (paper Sec. I: the triple-interaction n-body
// problem and the simplex-shaped outputs of pair problems).  Output E[p] for
// every triplet i < j < k < n, p the lexicographic rank
//   p(i,j,k) = C(n,3) - C(n-i,3) + T2(i,j) + (k - j - 1),
//   T2(i,j)  = (j-i-1)(n-1) - (j(j-1)/2 - i(i+1)/2)      (pairs (j', k) of row i
//              with j' < j), so T2(i, j+1) = T2(i, j) + (n - 1 - j).
// The energy of one triplet is written in the angle form itself,
//   E_t = nu (1 + 3 cos g_i cos g_j cos g_k) / (r1 r2 r3)^3
//       = nu (1 - 3 (a.b)(b.c)(c.a) R^2) R^3,   R = 1 / (r1 r2 r3),
// a = x_j - x_i, b = x_k - x_j, c = x_i - x_k (cos g_i = -(a.c) / (|a| |c|), ...),
// with the cosines taken from dot products of coordinate differences: each
// element is then accurate to a few units of FP32 rounding relative to its
// scale nu R^3.  (The squared-distance form used by the reductions forms
// 16 x squared area by cancellation, whose error grows with a triangle's aspect
// ratio; it is harmless in sums, not per element.)  About 21 FP32 operations per
// 4-byte store: the kernel is bound by the stores.
//
// Block: 256 threads own the 32^3 triplets of tile (X, Y, Z), X <= Y <= Z.
// (A second, tile-contiguous output layout is described at the kernel.)
//   1. positions of the three tiles -> LDS;
//   2. per pair of the sets (i,j), (i,k), (j,k) the difference vector and
//      d = 1/r -> LDS as one float4, stored [i][j], [i][k], [j][k]; d = 0 for a
//      pair out of order or past n (an invalid triplet computes 0; it is also
//      never stored);
//   3. lane kl of a half wave takes k = Z 32 + kl; half wave h takes i = X 32 +
//      h + 8 m (m < 4) and sweeps j over the Y tile: the 32 lanes store 32
//      consecutive k of one (i, j), one contiguous 128-byte run.
#include "smx_device.h"
#include "smx_internal.h"

namespace smx {

constexpr int kPackThreads = 256;

// TILED: the tile-contiguous layout instead of the lexicographic one.  Tile
// (X, Y, Z) of T3 owns the 32^3 floats starting at rank(X, Y, Z) * 32^3, rank =
// Z(Z+1)(Z+2)/6 + Y(Y+1)/2 + X (the tile's place in the listing by Z, Y, X);
// element (i, j, k) sits at offset 1024 (i mod 32) + 32 (j mod 32) + (k mod 32)
// inside it, and the tile's entries that are not triplets i < j < k < n hold
// 0.  Every tile is then one contiguous 128 KB run, written in full.
template <int MAP, bool STATS, bool TILED>
__global__ __launch_bounds__(kPackThreads) void at_packed_kernel(MapGeom g, const float *__restrict__ Xp,
                                                                 int64_t n, int64_t ldx, float nu,
                                                                 float *__restrict__ E,
                                                                 unsigned long long *sslots) {
    uint64_t lin;
    int TX, TY, TZ;
    if (!tile3_of<MAP, true>(g, lin, TX, TY, TZ)) return;
    constexpr int T = kTripTile, PS = T * T;
    __shared__ float4 Pos[3][T];
    // sets 0 (i,j): x_j - x_i; 1 (i,k): x_k - x_i; 2 (j,k): x_k - x_j; .w = 1/r
    __shared__ float4 Vp[3][PS];
    __shared__ unsigned long long sred[2][kPackThreads / kWave];

    const int t = threadIdx.x;
    const int64_t base[3] = {int64_t(TX) * T, int64_t(TY) * T, int64_t(TZ) * T};
    if (t < 3 * T) {
        const int tile = t >> 5, a = t & 31;
        const int64_t p = base[tile] + a;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (p < n) {
            v.x = Xp[p * ldx + 0];
            v.y = Xp[p * ldx + 1];
            v.z = Xp[p * ldx + 2];
        }
        Pos[tile][a] = v;
    }
    __syncthreads();

    // a tile with X < Y < Z wholly below n holds only valid triplets
    const bool interior = TX < TY && TY < TZ && base[2] + T <= n;
    {
        const int c = t & 31, r0 = t >> 5;
#pragma unroll
        for (int set = 0; set < 3; ++set) {
            const int ta = set == 2 ? 1 : 0, tb = set == 0 ? 1 : 2;  // row tile, column tile
            const float4 pb = Pos[tb][c];
            const int64_t gb = base[tb] + c;
#pragma unroll
            for (int it = 0; it < 4; ++it) {
                const int r = r0 + 8 * it;
                const float4 pa = Pos[ta][r];
                const float dx = pb.x - pa.x, dy = pb.y - pa.y, dz = pb.z - pa.z;
                const float sv = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                const int64_t ga = base[ta] + r;
                const bool valid = interior || (ga < gb && gb < n);
                Vp[set][r * T + c] = make_float4(dx, dy, dz, valid ? __builtin_amdgcn_rsqf(sv) : 0.f);
            }
        }
    }
    __syncthreads();

    const int kl = t & 31, h = t >> 5;
    const int64_t k = base[2] + kl;
    const int64_t c3 = n * (n - 1) * (n - 2) / 6;
    unsigned long long cnt = 0, cs = 0;
#pragma unroll 1
    for (int m = 0; m < 4; ++m) {
        const int il = h + 8 * m;
        const int64_t i = base[0] + il;
        const float4 vc = Vp[1][il * T + kl];  // x_k - x_i (= -c), 1/r_ik
        // element index of (i, j, k) minus k, at j = Y 32, advanced per j
        const int64_t ni = n - i, j0 = base[1];
        int64_t rowj = c3 - ni * (ni - 1) * (ni - 2) / 6 + (j0 - i - 1) * (n - 1) - (j0 * (j0 - 1) / 2 - i * (i + 1) / 2) -
                       j0 - 1;
        float *out = E + k;
        if (TILED) {
            const uint64_t Z = uint64_t(TZ), Y = uint64_t(TY);
            const uint64_t rank = Z * (Z + 1) * (Z + 2) / 6 + Y * (Y + 1) / 2 + uint64_t(TX);
            out = E + rank * uint64_t(T * T * T) + uint64_t(il * T * T + kl);
        }
#pragma unroll 4
        for (int jl = 0; jl < T; ++jl) {
            const int64_t j = j0 + jl;
            const float4 va = Vp[0][il * T + jl];  // a = x_j - x_i, 1/r_ij
            const float4 vb = Vp[2][jl * T + kl];  // b = x_k - x_j, 1/r_jk
            const float ab = __builtin_fmaf(va.z, vb.z, __builtin_fmaf(va.y, vb.y, va.x * vb.x));
            const float bc = __builtin_fmaf(vb.z, vc.z, __builtin_fmaf(vb.y, vc.y, vb.x * vc.x));
            const float ca = __builtin_fmaf(vc.z, va.z, __builtin_fmaf(vc.y, va.y, vc.x * va.x));
            const float R = va.w * (vb.w * vc.w);
            const float R2 = R * R;
            // (a.b)(b.c)(c.a) with c = -(x_k - x_i): the two sign flips cancel
            const float inner = __builtin_fmaf(-3.f, (ab * bc) * (ca * R2), 1.f);
            const float e = inner * (nu * (R2 * R));
            const bool ok = TILED ? (i < j && j < k && k < n)
                          : interior ? smx_check(i < j && j < k && k < n, kCheckStore) : (i < j && j < k && k < n);
            if (TILED)
                out[jl * T] = ok ? e : 0.f;
            else if (ok)
                out[rowj - jl] = e;
            if (STATS && ok) {
                ++cnt;
                cs += mix64(id_trip_lt(uint64_t(i), uint64_t(j), uint64_t(k)));
            }
            rowj += n - 1 - j;
        }
    }
    if (STATS) {
        const unsigned long long c = block_sum<unsigned long long, kPackThreads>(cnt, sred[0]);
        const unsigned long long hs = block_sum<unsigned long long, kPackThreads>(cs, sred[1]);
        if (t == 0) stats_add(sslots, lin, c, hs);
    }
}

template <int MAP, bool TILED>
static void go_packed(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float nu, float *E,
                      unsigned long long *sslots, hipStream_t s) {
    const dim3 grid = MAP == MAP_BBOX ? dim3(g.nb, g.nb, g.nb) : grid_for(g.G, kPackThreads);
    if (sslots)
        hipLaunchKernelGGL((at_packed_kernel<MAP, true, TILED>), grid, dim3(kPackThreads), 0, s, g, X, n, ldx, nu,
                           E, sslots);
    else
        hipLaunchKernelGGL((at_packed_kernel<MAP, false, TILED>), grid, dim3(kPackThreads), 0, s, g, X, n, ldx, nu,
                           E, sslots);
}

int launch_triplet_packed(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float nu, float *E,
                          unsigned long long *sslots, bool tiled, hipStream_t s) {
    const int kid = tiled ? K_TRIP_TILED : K_TRIP_PACKED;
    prof_begin(kid, s);
    for_each_launch(g, [&](auto M, const MapGeom &gg) {
        constexpr int MAPK = decltype(M)::value;
        if (tiled) go_packed<MAPK, true>(gg, X, n, ldx, nu, E, sslots, s);
        else go_packed<MAPK, false>(gg, X, n, ldx, nu, E, sslots, s);
    });
    prof_end(kid, s);
    return check_launch("triplet packed");
}

SMX_CHECK_READER(check_flags_tripack)

}  // namespace smx
