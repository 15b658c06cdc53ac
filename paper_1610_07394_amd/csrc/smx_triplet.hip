// Axilrod-Teller triplet energy and gradient on the 3-simplex, Lennard-Jones
// pairs on the 2-simplex (paper Sec. I: the triple-interaction n-body problem
// and the pair n-body problem).
//
// Per triplet i < j < k, with s1 = |x_j - x_i|^2, s2 = |x_k - x_j|^2,
// s3 = |x_i - x_k|^2 (law of cosines: cos g = t / (2 r r)):
//   E_t = nu (P - 3/8 T) P^(-5/2),   P = s1 s2 s3,   T = t1 t2 t3,
//   t1 = s3 - s1 - s2,  t2 = s1 - s2 - s3,  t3 = s2 - s3 - s1.
// The gradient never forms per-particle forces per triplet.  Because E depends
// on positions only through the pair terms, dE/dx_a = sum_b 2 W_ab (x_a - x_b)
// with W_ab = sum over triplets holding the pair {a, b} of dE_t/ds_ab.  So each
// triplet only adds three scalars:
//   dE_t/ds_p = nu (dP_p A' + dT_p B'),   A' = R - 5/2 N R / P,   B' = -3/8 R,
//   R = P^(-5/2), N = P - 3/8 T, dP = (s2 s3, s1 s3, s1 s2),
//   dT1 = 2 m2 - M, dT2 = 2 m3 - M, dT3 = 2 m1 - M,
//   m1 = t2 t3, m2 = t1 t3, m3 = t1 t2, M = m1 + m2 + m3.
// P^(-1/2) = d1 d2 d3 with d = 1/r per pair, so the triplet loop needs no
// square root: R = (d1 d2 d3)^5 and 1/P = (d1 d2 d3)^2.
//
// Block: 256 threads own the 32^3 triplets of tile (X, Y, Z), X <= Y <= Z.
//   1. positions of the three 32-particle tiles -> LDS;
//   2. the 3 x 32 x 32 pair terms s and d -> LDS; d = 0 for a pair that is out
//      of order (i >= j, j >= k, i >= k) or past n, which zeroes R for every
//      triplet containing it -- the simplex mask costs nothing per triplet and
//      diagonal tiles run the same code;
//   3. each thread runs 4 i x 4 j x 8 k (wave kb owns k in [8 kb, 8 kb + 8));
//      per k, the weights W_ik and W_jk are summed across lanes with DPP
//      (quad_perm within a quad, row_ror 4 / 8 across a row's quads) and each
//      entry is stored once into one of two half-wave planes; W_ij stays in
//      registers and each wave stores its own slice after the loop.  LDS
//      atomics cost far more than these shuffles on gfx950, and none remain;
//   4. pair weights -> forces on the 96 particles (64 pair terms each, two
//      threads per particle; the planes and slices are summed on read), FP64
//      atomics into the gradient;
//   5. energy: wave / block sums in FP64, one atomic into a spread slot.
#include "smx_device.h"
#include "smx_internal.h"

namespace smx {

constexpr int kTripThreads = 256;
constexpr int kTripLd = kTripTile + 4;  // LDS row stride (floats)

// DPP lane moves (all 64 lanes active): quad_perm xor 1 / xor 2 and
// row_ror 4 / 8 within a 16-lane row.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
// Sum over the 4 lanes of a quad; every lane gets the sum.
__device__ __forceinline__ float quad_allsum(float v) {
    v += dpp_mov<0xB1>(v);  // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);  // quad_perm [2,3,0,1]
    return v;
}
// Sum over lanes l, l+4, l+8, l+12 (mod 16) of a row; every lane gets the sum.
__device__ __forceinline__ float rowquads_allsum(float v) {
    v += dpp_mov<0x124>(v);  // row_ror:4
    v += dpp_mov<0x128>(v);  // row_ror:8
    return v;
}

template <int MAP, bool GRAD, bool STATS>
__global__ __launch_bounds__(kTripThreads, 3) void at_kernel(MapGeom g, const float *__restrict__ Xp, int64_t n,
                                                          int64_t ldx, float nu, double *__restrict__ G64,
                                                          double *__restrict__ eslots,
                                                          unsigned long long *sslots) {
    uint64_t lin;
    int TX, TY, TZ;
    if (!tile3_of<MAP, true>(g, lin, TX, TY, TZ)) return;

    constexpr int PS = kTripTile * kTripLd;
    __shared__ float4 Pos[3][kTripTile];
    // SD[0..2]: pair terms s ([i][j], [k][i], [k][j]); SD[3..5]: d = 1/r of the same
    // pairs.  After the triplet loop SD[0..3] hold the four per-wave slices of W_ij.
    __shared__ __attribute__((aligned(16))) float SD[6][PS];
    // per-k weights W_ik ([plane][k][i]) and W_jk ([plane][k][j]), two planes each
    __shared__ __attribute__((aligned(16))) float WZ[GRAD ? 4 : 1][GRAD ? PS : 1];
    __shared__ double red[kTripThreads / kWave];
    __shared__ unsigned long long sred[2][kTripThreads / kWave];

    const int t = threadIdx.x;
    const int64_t base[3] = {int64_t(TX) * kTripTile, int64_t(TY) * kTripTile, int64_t(TZ) * kTripTile};

    if (t < 3 * kTripTile) {
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

    // pair terms: set 0 rows i (X) cols j (Y); set 1 rows k (Z) cols i (X);
    // set 2 rows k (Z) cols j (Y).  Valid iff the pair is in triplet order
    // (i < j, i < k, j < k) and the larger index is < n.
    for (int e = t; e < 3 * kTripTile * kTripTile; e += kTripThreads) {
        const int set = e >> 10, r = (e >> 5) & 31, c = e & 31;
        const int ta = set == 0 ? 0 : 2, tb = set == 2 ? 1 : (set == 0 ? 1 : 0);
        const float4 pa = Pos[ta][r], pb = Pos[tb][c];
        const float dx = pb.x - pa.x, dy = pb.y - pa.y, dz = pb.z - pa.z;
        const float s = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
        const int64_t ga = base[ta] + r, gb = base[tb] + c;
        const bool valid = set == 0 ? (ga < gb && gb < n) : (gb < ga && ga < n);
        SD[set][r * kTripLd + c] = s;
        SD[3 + set][r * kTripLd + c] = valid ? __builtin_amdgcn_rsqf(s) : 0.f;
    }
    __syncthreads();

    // lane = 16 row + 4 q + e;  ib = 4 (row >> 1) + q,  jb = 4 (row & 1) + e;
    // the thread owns i in 4 ib + [0,4), j in 4 jb + [0,4), k in 8 kb + [0,8)
    const int lane = t & 63, kb = t >> 6, row = lane >> 4, q = (lane >> 2) & 3, el = lane & 3;
    const int ib = 4 * (row >> 1) + q, jb = 4 * (row & 1) + el;
    float s1[4][4], d1[4][4], w1[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const float4 sv = *reinterpret_cast<const float4 *>(&SD[0][(4 * ib + a) * kTripLd + 4 * jb]);
        const float4 dv = *reinterpret_cast<const float4 *>(&SD[3][(4 * ib + a) * kTripLd + 4 * jb]);
        s1[a][0] = sv.x; s1[a][1] = sv.y; s1[a][2] = sv.z; s1[a][3] = sv.w;
        d1[a][0] = dv.x; d1[a][1] = dv.y; d1[a][2] = dv.z; d1[a][3] = dv.w;
#pragma unroll
        for (int b = 0; b < 4; ++b) w1[a][b] = 0.f;
    }
    float e = 0.f;
    unsigned long long cnt = 0, cs = 0;

#pragma unroll 1
    for (int r = 0; r < 8; ++r) {
        const int k = 8 * kb + r;
        const float4 s3v = *reinterpret_cast<const float4 *>(&SD[1][k * kTripLd + 4 * ib]);
        const float4 d3v = *reinterpret_cast<const float4 *>(&SD[4][k * kTripLd + 4 * ib]);
        const float4 s2v = *reinterpret_cast<const float4 *>(&SD[2][k * kTripLd + 4 * jb]);
        const float4 d2v = *reinterpret_cast<const float4 *>(&SD[5][k * kTripLd + 4 * jb]);
        const float s3a[4] = {s3v.x, s3v.y, s3v.z, s3v.w}, d3a[4] = {d3v.x, d3v.y, d3v.z, d3v.w};
        const float s2a[4] = {s2v.x, s2v.y, s2v.z, s2v.w}, d2a[4] = {d2v.x, d2v.y, d2v.z, d2v.w};
        float w2[4] = {0.f, 0.f, 0.f, 0.f}, w3[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const float sa = s1[a][b], sb = s2a[b], sc = s3a[a];
                const float q23 = sb * sc;
                const float P = sa * q23;
                const float u = sa + sb + sc;
                const float t1 = __builtin_fmaf(2.f, sc, -u);
                const float t2 = __builtin_fmaf(2.f, sa, -u);
                const float t3 = __builtin_fmaf(2.f, sb, -u);
                const float Dd = d1[a][b] * (d2a[b] * d3a[a]);
                const float D2 = Dd * Dd;
                const float R = (D2 * D2) * Dd;
                if (!GRAD) {
                    const float T = t1 * t2 * t3;
                    const float N = __builtin_fmaf(-0.375f, T, P);
                    e = __builtin_fmaf(N, R, e);
                } else {
                    const float m1 = t2 * t3, m2 = t1 * t3, m3 = t1 * t2;
                    const float T = t1 * m1;
                    const float N = __builtin_fmaf(-0.375f, T, P);
                    const float NR = N * R;
                    e += NR;
                    const float A = __builtin_fmaf(-2.5f * NR, D2, R);
                    const float B = -0.375f * R;
                    const float M = m1 + m2 + m3;
                    const float dT1 = __builtin_fmaf(2.f, m2, -M);
                    const float dT2 = __builtin_fmaf(2.f, m3, -M);
                    const float dT3 = __builtin_fmaf(2.f, m1, -M);
                    const float q13 = sa * sc, q12 = sa * sb;
                    w1[a][b] = __builtin_fmaf(q23, A, __builtin_fmaf(dT1, B, w1[a][b]));
                    w2[b] = __builtin_fmaf(q13, A, __builtin_fmaf(dT2, B, w2[b]));
                    w3[a] = __builtin_fmaf(q12, A, __builtin_fmaf(dT3, B, w3[a]));
                }
                if (STATS) {
                    const int64_t gi = base[0] + 4 * ib + a, gj = base[1] + 4 * jb + b, gk = base[2] + k;
                    if (gi < gj && gj < gk && gk < n) {
                        ++cnt;
                        cs += mix64(id_trip_lt(uint64_t(gi), uint64_t(gj), uint64_t(gk)));
                    }
                }
            }
        if (GRAD) {
            // W_ik: sum the lane's partials over the quad (jb low bits); lane el
            // stores i = 4 ib + el into plane (row & 1).  W_jk: sum over the
            // row's quads (ib low bits); lane q stores j = 4 jb + q into plane
            // (row >> 1).  Each entry has exactly one writer: no atomics.
#pragma unroll
            for (int a = 0; a < 4; ++a) w3[a] = quad_allsum(w3[a]);
#pragma unroll
            for (int b = 0; b < 4; ++b) w2[b] = rowquads_allsum(w2[b]);
            const float v3 = el == 0 ? w3[0] : (el == 1 ? w3[1] : (el == 2 ? w3[2] : w3[3]));
            const float v2 = q == 0 ? w2[0] : (q == 1 ? w2[1] : (q == 2 ? w2[2] : w2[3]));
            WZ[row & 1][k * kTripLd + 4 * ib + el] = v3;
            WZ[2 + (row >> 1)][k * kTripLd + 4 * jb + q] = v2;
        }
    }

    // energy of the block, FP64 from the per-thread FP32 partials
    const double eb = block_sum<double, kTripThreads>(double(e), red);
    if (t == 0) atomicAdd(eslots + (lin % kSlots) * kSlotStride + 0, eb * double(nu));
    if (STATS) {
        const unsigned long long c = block_sum<unsigned long long, kTripThreads>(cnt, sred[0]);
        const unsigned long long h = block_sum<unsigned long long, kTripThreads>(cs, sred[1]);
        if (t == 0) stats_add(sslots, lin, c, h);
    }

    if (GRAD) {
        // every wave is past the triplet loop (block_sum synchronised): the pair
        // terms are dead, so SD[kb] takes this wave's slice of W_ij
#pragma unroll
        for (int a = 0; a < 4; ++a)
            *reinterpret_cast<float4 *>(&SD[kb][(4 * ib + a) * kTripLd + 4 * jb]) =
                make_float4(w1[a][0], w1[a][1], w1[a][2], w1[a][3]);
        __syncthreads();
        // particle p = t / 2 of the 96 (tile = p / 32), half h = t % 2:
        //   X (i): h0 sum_j W_ij (x_i - x_j),  h1 sum_k W_ik (x_i - x_k)
        //   Y (j): h0 sum_i W_ij (x_j - x_i),  h1 sum_k W_jk (x_j - x_k)
        //   Z (k): h0 sum_i W_ik (x_k - x_i),  h1 sum_j W_jk (x_k - x_j)
        if (t < 2 * 3 * kTripTile) {
            const int p = t >> 1, h = t & 1, tile = p >> 5, a = p & 31;
            const float4 me = Pos[tile][a];
            float gx = 0.f, gy = 0.f, gz = 0.f;
            int other;
            if (tile == 0) other = h == 0 ? 1 : 2;
            else if (tile == 1) other = h == 0 ? 0 : 2;
            else other = h == 0 ? 0 : 1;
#pragma unroll 4
            for (int b = 0; b < kTripTile; ++b) {
                float wgt;
                if (tile == 0 && h == 0) {
                    const int o = a * kTripLd + b;
                    wgt = (SD[0][o] + SD[1][o]) + (SD[2][o] + SD[3][o]);
                } else if (tile == 1 && h == 0) {
                    const int o = b * kTripLd + a;
                    wgt = (SD[0][o] + SD[1][o]) + (SD[2][o] + SD[3][o]);
                } else if ((tile == 0 && h == 1) || (tile == 2 && h == 0)) {
                    const int o = tile == 0 ? b * kTripLd + a : a * kTripLd + b;  // W_ik stored [k][i]
                    wgt = WZ[0][o] + WZ[1][o];
                } else {
                    const int o = tile == 1 ? b * kTripLd + a : a * kTripLd + b;  // W_jk stored [k][j]
                    wgt = WZ[2][o] + WZ[3][o];
                }
                const float4 ot = Pos[other][b];
                gx = __builtin_fmaf(wgt, me.x - ot.x, gx);
                gy = __builtin_fmaf(wgt, me.y - ot.y, gy);
                gz = __builtin_fmaf(wgt, me.z - ot.z, gz);
            }
            gx += __shfl_xor(gx, 1, kWave);
            gy += __shfl_xor(gy, 1, kWave);
            gz += __shfl_xor(gz, 1, kWave);
            const int64_t gp = base[tile] + a;
            if (h == 0 && gp < n) {
                const double sc = 2.0 * double(nu);
                atomicAdd(G64 + 3 * gp + 0, sc * double(gx));
                atomicAdd(G64 + 3 * gp + 1, sc * double(gy));
                atomicAdd(G64 + 3 * gp + 2, sc * double(gz));
            }
        }
    }
}

template <int MAP, bool GRAD>
static void go_at(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float nu, double *G64,
                  double *eslots, unsigned long long *sslots, hipStream_t s) {
    const dim3 grid = MAP == MAP_BBOX ? dim3(g.nb, g.nb, g.nb) : grid_for(g.G, kTripThreads);
    if (sslots)
        hipLaunchKernelGGL((at_kernel<MAP, GRAD, true>), grid, dim3(kTripThreads), 0, s, g, X, n, ldx, nu,
                           G64, eslots, sslots);
    else
        hipLaunchKernelGGL((at_kernel<MAP, GRAD, false>), grid, dim3(kTripThreads), 0, s, g, X, n, ldx, nu,
                           G64, eslots, sslots);
}

int launch_triplet(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float nu, bool grad,
                   double *G64, double *eslots, unsigned long long *sslots, hipStream_t s) {
    const int kid = grad ? K_TRIP_GRAD : K_TRIP_ENERGY;
    prof_begin(kid, s);
    map_switch(int(g.map), [&](auto M) {
        constexpr int MAPK = decltype(M)::value;
        if (grad) go_at<MAPK, true>(g, X, n, ldx, nu, G64, eslots, sslots, s);
        else go_at<MAPK, false>(g, X, n, ldx, nu, G64, eslots, sslots, s);
    });
    prof_end(kid, s);
    return check_launch(grad ? "triplet energy+grad" : "triplet energy");
}

// ---------------------------------------------------------------- Lennard-Jones
// Tile 64 x 64 of pairs i < j; thread (tx, ty) owns rows ty + 16 r and columns
// tx + 16 c.  phi(s) = 4 eps (u^6 - u^3), u = sigma^2 / s; dphi/ds =
// 4 eps (3 u^3 - 6 u^6) / s.  Inside the cutoff iff s < fl(rc^2) with s
// formed exactly as fl(fma(dz,dz, fma(dy,dy, dx*dx))).
constexpr int kLjThreads = 256;

template <int MAP, bool STATS>
__global__ __launch_bounds__(kLjThreads) void lj_kernel(MapGeom g, const float *__restrict__ Xp, int64_t n,
                                                        int64_t ldx, float eps, float sig2, float rc2,
                                                        double *__restrict__ G64, double *__restrict__ eslots,
                                                        unsigned long long *sslots) {
    uint64_t lin;
    int TX, TY;
    if (!tile2_of<MAP, true>(g, lin, TX, TY)) return;
    __shared__ float4 Pi[kLjTile], Pj[kLjTile];
    __shared__ float Fi[kLjTile][3], Fj[kLjTile][3];
    __shared__ double red[kLjThreads / kWave];
    __shared__ unsigned long long sred[2][kLjThreads / kWave];
    const int t = threadIdx.x;
    const int64_t i0 = int64_t(TX) * kLjTile, j0 = int64_t(TY) * kLjTile;
    if (t < 2 * kLjTile) {
        const int a = t & (kLjTile - 1);
        const int64_t p = (t < kLjTile ? i0 : j0) + a;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (p < n) {
            v.x = Xp[p * ldx + 0];
            v.y = Xp[p * ldx + 1];
            v.z = Xp[p * ldx + 2];
        }
        if (t < kLjTile) Pi[a] = v;
        else Pj[a] = v;
    }
    for (int e = t; e < 2 * 3 * kLjTile; e += kLjThreads) {
        if (e < 3 * kLjTile) (&Fi[0][0])[e] = 0.f;
        else (&Fj[0][0])[e - 3 * kLjTile] = 0.f;
    }
    __syncthreads();
    const int tx = t & 15, ty = t >> 4;
    float e = 0.f;
    float gi[4][3], gj[4][3];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) gi[r][q] = gj[r][q] = 0.f;
    unsigned long long cnt = 0, cs = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float4 a = Pi[ty + 16 * r];
        const int64_t i = i0 + ty + 16 * r;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const float4 b = Pj[tx + 16 * c];
            const int64_t j = j0 + tx + 16 * c;
            const float dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
            const float s = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
            const bool pair = i < j && j < n;
            const bool in = pair && s < rc2;
            const float inv = in ? 1.0f / s : 0.f;
            const float u = sig2 * inv;
            const float u3 = u * u * u;
            const float u6 = u3 * u3;
            e += 4.f * eps * (u6 - u3);
            // dphi/ds, then dE/dx_i = -2 w (x_j - x_i), dE/dx_j = +2 w (x_j - x_i)
            const float wgt = 4.f * eps * (3.f * u3 - 6.f * u6) * inv;
            gi[r][0] -= wgt * dx; gi[r][1] -= wgt * dy; gi[r][2] -= wgt * dz;
            gj[c][0] += wgt * dx; gj[c][1] += wgt * dy; gj[c][2] += wgt * dz;
            if (STATS && pair) {
                ++cnt;
                cs += mix64(id_pair_lt(uint64_t(i), uint64_t(j)));
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            atomicAdd(&Fi[ty + 16 * r][q], gi[r][q]);
            atomicAdd(&Fj[tx + 16 * r][q], gj[r][q]);
        }
    const double eb = block_sum<double, kLjThreads>(double(e), red);
    if (t == 0) atomicAdd(eslots + (lin % kSlots) * kSlotStride + 1, eb);
    if (STATS) {
        const unsigned long long c = block_sum<unsigned long long, kLjThreads>(cnt, sred[0]);
        const unsigned long long h = block_sum<unsigned long long, kLjThreads>(cs, sred[1]);
        if (t == 0) stats_add(sslots, lin, c, h);
    }
    __syncthreads();
    if (t < 2 * kLjTile) {
        const int a = t & (kLjTile - 1);
        const int64_t p = (t < kLjTile ? i0 : j0) + a;
        if (p < n) {
            const float *f = t < kLjTile ? Fi[a] : Fj[a];
            atomicAdd(G64 + 3 * p + 0, 2.0 * double(f[0]));
            atomicAdd(G64 + 3 * p + 1, 2.0 * double(f[1]));
            atomicAdd(G64 + 3 * p + 2, 2.0 * double(f[2]));
        }
    }
}

template <int MAP>
static void go_lj(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float eps, float sig2,
                  float rc2, double *G64, double *eslots, unsigned long long *sslots, hipStream_t s) {
    const dim3 grid = MAP == MAP_BBOX ? dim3(g.nb, g.nb, 1) : grid_for(g.G, kLjThreads);
    if (sslots)
        hipLaunchKernelGGL((lj_kernel<MAP, true>), grid, dim3(kLjThreads), 0, s, g, X, n, ldx, eps, sig2, rc2,
                           G64, eslots, sslots);
    else
        hipLaunchKernelGGL((lj_kernel<MAP, false>), grid, dim3(kLjThreads), 0, s, g, X, n, ldx, eps, sig2, rc2,
                           G64, eslots, sslots);
}

int launch_lj(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float eps, float sigma,
              float rc2, double *G64, double *eslots, unsigned long long *sslots, hipStream_t s) {
    prof_begin(K_LJ, s);
    const float sig2 = sigma * sigma;
    map_switch(int(g.map), [&](auto M) { go_lj<decltype(M)::value>(g, X, n, ldx, eps, sig2, rc2, G64, eslots, sslots, s); });
    prof_end(K_LJ, s);
    return check_launch("lennard-jones");
}

// ---------------------------------------------------------------- finalize
__global__ void energy_finalize_kernel(const double *eslots, double *E) {
    __shared__ double red[2][kSlots / kWave];
    const int t = threadIdx.x;  // kSlots threads
    const double a = block_sum<double, kSlots>(eslots[t * kSlotStride + 0], red[0]);
    const double b = block_sum<double, kSlots>(eslots[t * kSlotStride + 1], red[1]);
    if (t == 0) {
        E[0] = a + b;
        E[1] = a;
        E[2] = b;
    }
}

int launch_energy_finalize(const double *eslots, double *E, hipStream_t s) {
    prof_begin(K_FINALIZE, s);
    hipLaunchKernelGGL(energy_finalize_kernel, dim3(1), dim3(kSlots), 0, s, eslots, E);
    prof_end(K_FINALIZE, s);
    return check_launch("energy finalize");
}

__global__ void grad_finalize_kernel(const double *G64, int64_t m, const double *gradE, float *out) {
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const double sc = gradE != nullptr ? gradE[0] : 1.0;
    out[q] = float(sc * G64[q]);
}

__global__ void scale_grad_kernel(const float *G, int64_t m, const double *gradE, float *out) {
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q < m) out[q] = float(gradE[0] * double(G[q]));
}

int launch_scale_grad(const float *G, int64_t n, const double *gradE, float *out, hipStream_t s) {
    const int64_t m = 3 * n;
    prof_begin(K_FINALIZE, s);
    hipLaunchKernelGGL(scale_grad_kernel, dim3(uint32_t((m + 255) / 256)), dim3(256), 0, s, G, m, gradE, out);
    prof_end(K_FINALIZE, s);
    return check_launch("scale grad");
}

int launch_grad_finalize(const double *G64, int64_t n, const double *gradE, float *out, hipStream_t s) {
    const int64_t m = 3 * n;
    prof_begin(K_FINALIZE, s);
    hipLaunchKernelGGL(grad_finalize_kernel, dim3(uint32_t((m + 255) / 256)), dim3(256), 0, s, G64, m,
                       gradE, out);
    prof_end(K_FINALIZE, s);
    return check_launch("grad finalize");
}

}  // namespace smx
