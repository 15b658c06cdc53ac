// Axilrod-Teller triplet energy and gradient on the 3-simplex, Lennard-Jones
// pairs on the 2-simplex (paper Sec. I: the triple-interaction n-body problem
// and the pair n-body problem).
//
// Per triplet i < j < k, with s1 = |x_j - x_i|^2, s2 = |x_k - x_j|^2,
// s3 = |x_i - x_k|^2 (law of cosines: cos g = t / (2 r r)):
//   E_t = nu (P - 3/8 T) P^(-5/2),   P = s1 s2 s3,   T = t1 t2 t3,
//   t1 = s3 - s1 - s2,  t2 = s1 - s2 - s3,  t3 = s2 - s3 - s1.
// The kernel evaluates the same quantity in symmetric-function form.  With
// u = s1 + s2 + s3 and g = 4 s2 s3 - (s1 - s2 - s3)^2 (= 16 x squared triangle
// area, symmetric in the three pairs), T = t1 t2 t3 = 8 P - u g, so
//   P - 3/8 T = 3/8 u g - 2 P,
// and its derivative with respect to one pair term s_p, together with
// dP^(-5/2)/ds_p = -5/2 P^(-5/2) / s_p, gives
//   dE_t/ds_p = 3/8 nu R (K - 4 u s_p - Q / s_p),
//   R = P^(-5/2),  K = g + 2 u^2,  Q = 5/2 u g - 8 P,
//   E_t = 1/4 nu R (Q - u g).
// Per pair the kernel keeps s, -4 s and d^5 (d = 1/r), so R = d1^5 d2^5 d3^5
// and the triplet loop has no square root, division or per-triplet power.
// The loop accumulates s_p dE_t/ds_p = 3/8 nu R (s_p (K - 4 u s_p) - Q)
// (K - 4 u s_1 as g - 2 u t2) and the sums are scaled by 1/s_p once per pair
// after the loop.  E_t is homogeneous of
// degree -9/2 in the pair terms, so (Euler) sum_p s_p dE_t/ds_p = -9/2 E_t:
// the energy is read off the same sums, E_t = -(nu / 12) R sum_p x_p with
// x_p = s_p (K - 4 u s_p) - Q.  About 22 FP32 operations per triplet give the
// energy and all three weights (8 P from a register copy of 2 s_ij).
// The gradient never forms per-particle forces per triplet.  Because E depends
// on positions only through the pair terms, dE/dx_a = sum_b 2 W_ab (x_a - x_b)
// with W_ab = sum over triplets holding the pair {a, b} of dE_t/ds_ab.  So each
// triplet only adds three scalars.
//
// Block: 256 threads own the 32^3 triplets of tile (X, Y, Z), X <= Y <= Z, one
// tile after another: the grid is persistent (at most kAtPersistBlocks blocks;
// kAtPersistBlocksG32 when the groups below hold 32 ids),
// the logical ids are dealt out in groups of R = 2^r consecutive ids (block b
// taking groups b, b + grid, ...: every block samples the whole parallel space,
// so blocks take equal time; R = 1 for the maps with many empty ids), and each
// tile's positions are loaded while the previous tile's triplets run, so a
// block no longer starts with a global load (with one block per tile the
// kernel took 64-65 ms, persistent 55 ms, before the changes below).  Consecutive
// ids of every map here move one tile index and keep the other two (lambda3
// walks w_x fastest: a Pi3 row changes X on one side of its fold and Z on the
// other; the bounding box and the linear listing change X), so inside a group
// a particle tile's forces are summed in registers while its index stays and
// go to the gradient once when it changes.
//   1. positions of the three 32-particle tiles -> LDS;
//   2. the 3 x 32 x 32 pair terms s, -4 s, d^5 -> LDS; d^5 = 0 for a pair that
//      is out of order (i >= j, j >= k, i >= k) or past n, which zeroes R for
//      every triplet containing it -- the simplex mask costs nothing per
//      triplet and diagonal tiles run the same code;
//   3. each thread runs 4 i x 4 j x 8 k (wave kb owns k in [8 kb, 8 kb + 8));
//      the (i, j) pair terms stay in registers for the whole loop; per k, the
//      weights W_ik and W_jk are summed across lanes with DPP (quad_perm
//      within a quad, row_ror 4 / 8 across a row's quads) and each entry is
//      stored once into one of two half-wave planes; W_ij stays in registers
//      and each wave stores its own slice after the loop.  LDS atomics cost
//      far more than these shuffles on gfx950, and none remain;
//   4. the planes and slices are summed into one plane per pair set, scaled
//      by 1/s_p (0 outside the simplex), and each is also stored transposed,
//      so every particle reads its weights along a row; pair weights -> forces on the 96 particles (one wave per tile,
//      half a wave per pair set), x_a sum_b W_ab - sum_b W_ab x_b, FP64
//      atomics into the gradient;
//   5. energy: wave / block sums in FP64, one atomic into a spread slot.
#include <type_traits>

#include "smx_device.h"
#include "smx_internal.h"

namespace smx {

constexpr int kTripThreads = 256;
// persistent grid of the triplet kernels: about 32 blocks per resident block
// slot (256 CUs x 3 blocks), and a prime, so that a block's ids or groups
// b, b + grid, ... do not keep to one position of the parallel space's rows
// (which are powers of two or nb long).
constexpr int kAtPersistBlocks = 24571;
// grid cap of the launches that deal groups of 32 (the largest ones: about one
// group per block, 128 blocks per slot, also a prime): 53.3 -> 52.7 ms at
// n = 8192 against 24571 blocks; smaller launches keep the cap above
constexpr int kAtPersistBlocksG32 = 98299;
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
                                                          unsigned long long *sslots, int grp_lg) {
    // Plane stride: 16 floats of padding put consecutive planes 16 of the 32 LDS
    // banks apart, so the two half-wave weight planes that one store of the k
    // loop writes (lanes 0-15 and 16-31 at the same offsets) share no bank.
    constexpr int PS = kTripTile * kTripLd + 16;
    // LDS planes of PS floats.  Pair sets: ij (rows i, cols j), ki (rows k,
    // cols i), kj (rows k, cols j).
    //   GRAD:  0 s_ki, 1 s_kj, 2 m4_ki, 3 m4_kj, 4 d5_ki, 5 d5_kj (m4 = -4 s);
    //          6..9: s_ij, d5_ij until every thread holds its (i, j) terms in
    //          registers, then the per-k weight planes W_ik (6, 7) and W_jk
    //          (8, 9), stored [k][i] and [k][j].  After the loop 2..5 take the
    //          W_ij slices; then W_ij [i][j] -> 2, W_ik [k][i] -> 6,
    //          W_jk [k][j] -> 8 and their transposes -> 3, 7, 9.
    //   energy only: 0 s_ki, 1 s_kj, 2 s_ij, 3 d5_ij, 4 d5_ki, 5 d5_kj.
    constexpr int NP = GRAD ? 10 : 6;
    constexpr int S_KI = 0, S_KJ = 1, M4_KI = 2, M4_KJ = 3, D5_KI = 4, D5_KJ = 5;
    constexpr int S_IJ = GRAD ? 6 : 2, D5_IJ = GRAD ? 7 : 3, W_IK = 6, W_JK = 8;
    __shared__ float4 Pos[3][kTripTile];
    __shared__ __attribute__((aligned(16))) float L[NP * PS];
    __shared__ double red[kTripThreads / kWave];
    __shared__ unsigned long long sred[2][kTripThreads / kWave];
    auto plane = [&](int i) -> float * { return L + i * PS; };

    const int t = threadIdx.x;
    // persistent blocks: block b takes the ids of groups b, b + nblk, ... in
    // order; the next tile's positions are loaded while the current tile's
    // triplets run
    const uint64_t nblk = uint64_t(gridDim.x) * gridDim.y, R = uint64_t(1) << grp_lg;
    uint64_t id = (uint64_t(blockIdx.y) * gridDim.x + blockIdx.x) << grp_lg;
    auto advance = [&](uint64_t i) -> uint64_t {  // the block's next id
        ++i;
        return (i & (R - 1)) ? i : i + (nblk - 1) * R;
    };
    auto next_valid = [&](uint64_t &i, uint64_t &l, int &x, int &y, int &z) -> bool {
        for (; i < g.G; i = advance(i))
            if (tile3_of_id<MAP>(g, uint32_t(i), l, x, y, z)) return true;
        return false;
    };
    // forces on the particles of this wave's tile role (wave 0 X, 1 Y, 2 Z),
    // lanes 0-31, summed while the role's tile index stays (FP64)
    double fx = 0.0, fy = 0.0, fz = 0.0;
    auto load_pos = [&](int x, int y, int z) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (t < 3 * kTripTile) {
            const int tile = t >> 5, a = t & 31;
            const int64_t p = int64_t(tile == 0 ? x : (tile == 1 ? y : z)) * kTripTile + a;
            if (p < n) {
                v.x = Xp[p * ldx + 0];
                v.y = Xp[p * ldx + 1];
                v.z = Xp[p * ldx + 2];
            }
        }
        return v;
    };
    uint64_t lin;
    int TX, TY, TZ;
    if (!next_valid(id, lin, TX, TY, TZ)) return;
    float4 pv = load_pos(TX, TY, TZ);
    while (true) {
        const int64_t base[3] = {int64_t(TX) * kTripTile, int64_t(TY) * kTripTile, int64_t(TZ) * kTripTile};
        if (t < 3 * kTripTile) Pos[t >> 5][t & 31] = pv;
        __syncthreads();
        uint64_t nid = advance(id), nlin = 0;
        int NX = 0, NY = 0, NZ = 0;
        const bool more = next_valid(nid, nlin, NX, NY, NZ);
        const float4 pnext = more ? load_pos(NX, NY, NZ) : make_float4(0.f, 0.f, 0.f, 0.f);

        // pair terms: set 0 rows i (X) cols j (Y); set 1 rows k (Z) cols i (X);
        // set 2 rows k (Z) cols j (Y).  Valid iff the pair is in triplet order
        // (i < j, i < k, j < k) and the larger index is < n.  Thread t takes
        // column t % 32 and rows t / 32 + 8 it of every set; indices fit 32 bits
        // (n < 2^31, tile bases < n + 32).  An interior tile (X < Y < Z, all of it
        // below n: nearly every block) has only valid pairs and skips the test.
        const bool interior = TX < TY && TY < TZ && base[2] + kTripTile <= n;
        auto pair_terms = [&](auto full) {
            constexpr bool FULL = decltype(full)::value;
            const int c = t & 31, r0 = t >> 5;
            const uint32_t un = uint32_t(n);
            const uint32_t bt[3] = {uint32_t(base[0]), uint32_t(base[1]), uint32_t(base[2])};
#pragma unroll
            for (int set = 0; set < 3; ++set) {
                const int ta = set == 0 ? 0 : 2, tb = set == 2 ? 1 : (set == 0 ? 1 : 0);
                const float4 pb = Pos[tb][c];
                const uint32_t gb = bt[tb] + uint32_t(c);
#pragma unroll
                for (int it = 0; it < 4; ++it) {
                    const int r = r0 + 8 * it;
                    const float4 pa = Pos[ta][r];
                    const float dx = pb.x - pa.x, dy = pb.y - pa.y, dz = pb.z - pa.z;
                    const float sv = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
                    const uint32_t ga = bt[ta] + uint32_t(r);
                    const bool valid = FULL || (set == 0 ? (ga < gb && gb < un) : (gb < ga && ga < un));
                    const float d = valid ? __builtin_amdgcn_rsqf(sv) : 0.f;
                    const float rs = d * d;
                    const int o = r * kTripLd + c;
                    plane(set == 0 ? S_IJ : S_KI + set - 1)[o] = sv;
                    plane(set == 0 ? D5_IJ : D5_KI + set - 1)[o] = (rs * rs) * d;
                    if (GRAD && set != 0) plane(M4_KI + set - 1)[o] = -4.f * sv;
                }
            }
        };
        if (interior) pair_terms(std::true_type{});
        else pair_terms(std::false_type{});
        __syncthreads();

        // lane = 16 row + 4 q + e;  ib = 4 (row >> 1) + q,  jb = 4 (row & 1) + e;
        // the thread owns i in 4 ib + [0,4), j in 4 jb + [0,4), k in 8 kb + [0,8)
        const int lane = t & 63, row = lane >> 4, q = (lane >> 2) & 3, el = lane & 3;
        const int kb = __builtin_amdgcn_readfirstlane(t >> 6);  // wave index
        const int ib = 4 * (row >> 1) + q, jb = 4 * (row & 1) + el;
        float s1[4][4], f1[4][4], w1[4][4], s1x2[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int o = (4 * ib + a) * kTripLd + 4 * jb;
            const float4 sv = *reinterpret_cast<const float4 *>(plane(S_IJ) + o);
            const float4 fv = *reinterpret_cast<const float4 *>(plane(D5_IJ) + o);
            s1[a][0] = sv.x; s1[a][1] = sv.y; s1[a][2] = sv.z; s1[a][3] = sv.w;
            f1[a][0] = fv.x; f1[a][1] = fv.y; f1[a][2] = fv.z; f1[a][3] = fv.w;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                w1[a][b] = 0.f;
                s1x2[a][b] = s1[a][b] + s1[a][b];
            }
        }
        // the (i, j) planes become the per-k weight planes
        if (GRAD) __syncthreads();
        float e = 0.f;
        unsigned long long cnt = 0, cs = 0;

#pragma unroll 1
        for (int r = 0; r < 8; ++r) {
            const int k = 8 * kb + r;
            const int oi = k * kTripLd + 4 * ib, oj = k * kTripLd + 4 * jb;
            const float4 s3v = *reinterpret_cast<const float4 *>(plane(S_KI) + oi);
            const float4 f3v = *reinterpret_cast<const float4 *>(plane(D5_KI) + oi);
            const float4 s2v = *reinterpret_cast<const float4 *>(plane(S_KJ) + oj);
            const float4 f2v = *reinterpret_cast<const float4 *>(plane(D5_KJ) + oj);
            const float s3a[4] = {s3v.x, s3v.y, s3v.z, s3v.w}, f3a[4] = {f3v.x, f3v.y, f3v.z, f3v.w};
            const float s2a[4] = {s2v.x, s2v.y, s2v.z, s2v.w}, f2a[4] = {f2v.x, f2v.y, f2v.z, f2v.w};
            float m3a[4], m2a[4];  // -4 s
            if (GRAD) {
                const float4 m3v = *reinterpret_cast<const float4 *>(plane(M4_KI) + oi);
                const float4 m2v = *reinterpret_cast<const float4 *>(plane(M4_KJ) + oj);
                m3a[0] = m3v.x; m3a[1] = m3v.y; m3a[2] = m3v.z; m3a[3] = m3v.w;
                m2a[0] = m2v.x; m2a[1] = m2v.y; m2a[2] = m2v.z; m2a[3] = m2v.w;
            } else {
#pragma unroll
                for (int b = 0; b < 4; ++b) m2a[b] = -4.f * s2a[b];
            }
            float w2[4] = {0.f, 0.f, 0.f, 0.f}, w3[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const float sa = s1[a][b], sb = s2a[b], sc = s3a[a];
                    const float v = sb + sc;
                    const float t2n = v - sa;                   // -t2
                    const float u = sa + v;
                    const float q4 = -(m2a[b] * sc);            // 4 s2 s3
                    const float gg = __builtin_fmaf(-t2n, t2n, q4);  // g
                    const float y = u * gg;
                    const float P8 = s1x2[a][b] * q4;           // 8 P
                    const float R = f1[a][b] * (f2a[b] * f3a[a]);
                    if (!GRAD) {
                        // 4 (P - 3/8 T) = 3/2 u g - 8 P
                        e = __builtin_fmaf(__builtin_fmaf(1.5f, y, -P8), R, e);
                    } else {
                        const float nQ = __builtin_fmaf(-2.5f, y, P8);  // -Q = 8 P - 5/2 u g
                        const float tu = u + u;
                        const float K = __builtin_fmaf(tu, u, gg);
                        // s_p (K - 4 u s_p) - Q;  K - 4 u s_1 = g - 2 u t2
                        const float x1 = __builtin_fmaf(sa, __builtin_fmaf(tu, t2n, gg), nQ);
                        const float x2 = __builtin_fmaf(sb, __builtin_fmaf(u, m2a[b], K), nQ);
                        const float x3 = __builtin_fmaf(sc, __builtin_fmaf(u, m3a[a], K), nQ);
                        w1[a][b] = __builtin_fmaf(R, x1, w1[a][b]);
                        w2[b] = __builtin_fmaf(R, x2, w2[b]);
                        w3[a] = __builtin_fmaf(R, x3, w3[a]);
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
                // (row >> 1).  Each entry has exactly one writer: no atomics.  The
                // sums carry a factor s_p, removed after the loop.
#pragma unroll
                for (int a = 0; a < 4; ++a) w3[a] = quad_allsum(w3[a]);
#pragma unroll
                for (int b = 0; b < 4; ++b) w2[b] = rowquads_allsum(w2[b]);
                // selects on the index bits (an equality chain becomes a branch
            // per case, which costs registers the persistent loop needs)
            const float v3 = (el & 2) ? ((el & 1) ? w3[3] : w3[2]) : ((el & 1) ? w3[1] : w3[0]);
                const float v2 = (q & 2) ? ((q & 1) ? w2[3] : w2[2]) : ((q & 1) ? w2[1] : w2[0]);
                plane(W_IK + (row & 1))[oi + el] = v3;
                plane(W_JK + (row >> 1))[oj + q] = v2;
            }
        }

        // energy of the block, FP64 from the per-thread FP32 partials: sums of
        // 4 (P - 3/8 T) R (energy only) or of R (x_1 + x_2 + x_3) = -12 (P - 3/8 T) R
        // (with the gradient: the R x_1 sums here, the R x_2 and R x_3 sums from
        // the weight planes after the loop)
        if (GRAD) {
#pragma unroll
            for (int a = 0; a < 4; ++a) e += (w1[a][0] + w1[a][1]) + (w1[a][2] + w1[a][3]);
        }
        if (!GRAD) {
            const double eb = block_sum<double, kTripThreads>(double(e), red);
            if (t == 0) atomicAdd(eslots + (lin % kSlots) * kSlotStride + 0, eb * (0.25 * double(nu)));
        }
        if (STATS) {
            const unsigned long long c = block_sum<unsigned long long, kTripThreads>(cnt, sred[0]);
            const unsigned long long h = block_sum<unsigned long long, kTripThreads>(cs, sred[1]);
            if (t == 0) stats_add(sslots, lin, c, h);
        }

        if (GRAD) {
            // every wave is past the triplet loop: the -4 s and d^5 planes (2..5)
            // are dead, so plane 2 + kb takes this wave's slice of W_ij (its sums
            // carry s_ij: divide, 0 outside the simplex)
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 4; ++a) {
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    w1[a][b] = (interior || f1[a][b] != 0.f) ? w1[a][b] * __builtin_amdgcn_rcpf(s1[a][b]) : 0.f;
                *reinterpret_cast<float4 *>(plane(2 + kb) + (4 * ib + a) * kTripLd + 4 * jb) =
                    make_float4(w1[a][0], w1[a][1], w1[a][2], w1[a][3]);
            }
            __syncthreads();
            // one plane per pair set: W_ij -> plane 2, W_ik -> 6, W_jk -> 8 (in
            // place), the last two divided by s (a pair outside the simplex has
            // zero sums; s = 0 only for such pairs)
            for (int o = t; o < kTripTile * kTripTile; o += kTripThreads) {
                const int x = (o >> 5) * kTripLd + (o & 31);
                plane(2)[x] = (plane(2)[x] + plane(3)[x]) + (plane(4)[x] + plane(5)[x]);
                const float ski = plane(S_KI)[x], skj = plane(S_KJ)[x];
                const float rik = plane(W_IK)[x] + plane(W_IK + 1)[x], rjk = plane(W_JK)[x] + plane(W_JK + 1)[x];
                e += rik + rjk;  // the R x_3 and R x_2 sums of the energy
                plane(W_IK)[x] = ski > 0.f ? rik * __builtin_amdgcn_rcpf(ski) : 0.f;
                plane(W_JK)[x] = skj > 0.f ? rjk * __builtin_amdgcn_rcpf(skj) : 0.f;
            }
            const double eb = block_sum<double, kTripThreads>(double(e), red);  // synchronises the block
            if (t == 0) atomicAdd(eslots + (lin % kSlots) * kSlotStride + 0, eb * (-double(nu) / 12.0));
            // transposes: W_ji [j][i] -> 3, W_ik [i][k] -> 7, W_jk [j][k] -> 9.  A
            // half-wave takes one diagonal d of the plane, lane r the element
            // (r, (r + d) mod 32): the banks of the read (5 r + d) and of the
            // transposed store (5 r + 4 d, mod 32) are distinct across its 32 lanes.
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int r = t & 31, c = (r + (t >> 5) + 8 * m) & 31;
                const int x = r * kTripLd + c, xt = c * kTripLd + r;
                plane(3)[xt] = plane(2)[x];
                plane(W_IK + 1)[xt] = plane(W_IK)[x];
                plane(W_JK + 1)[xt] = plane(W_JK)[x];
            }
            __syncthreads();
            // wave T < 3 takes tile T; lane = 32 h + a: particle a, pair set h.
            //   X (i): h0 W_ij [i][j] (plane 2) with j,  h1 W_ik [i][k] (7) with k
            //   Y (j): h0 W_ji [j][i] (3) with i,        h1 W_jk [j][k] (9) with k
            //   Z (k): h0 W_ki [k][i] (6) with i,        h1 W_kj [k][j] (8) with j
            // dE/dx_a = 2 nu sum_b W_ab (x_a - x_b) = 2 nu (x_a sum_b W_ab - sum_b W_ab x_b)
            if (kb < 3) {
                const int tile = kb, a = lane & 31, h = lane >> 5;
                const int pl = tile == 0 ? (h == 0 ? 2 : W_IK + 1)
                                         : (tile == 1 ? (h == 0 ? 3 : W_JK + 1) : (h == 0 ? W_IK : W_JK));
                const int other = tile == 0 ? 1 + h : (tile == 1 ? 2 * h : h);
                const float *W = plane(pl) + a * kTripLd;
                float ws = 0.f, wx = 0.f, wy = 0.f, wz = 0.f;
#pragma unroll 2
                for (int b = 0; b < kTripTile; b += 4) {
                    const float4 w4 = *reinterpret_cast<const float4 *>(W + b);
                    const float wv[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const float4 ot = Pos[other][b + c];
                        ws += wv[c];
                        wx = __builtin_fmaf(wv[c], ot.x, wx);
                        wy = __builtin_fmaf(wv[c], ot.y, wy);
                        wz = __builtin_fmaf(wv[c], ot.z, wz);
                    }
                }
                const float4 me = Pos[tile][a];
                float gx = __builtin_fmaf(me.x, ws, -wx), gy = __builtin_fmaf(me.y, ws, -wy),
                      gz = __builtin_fmaf(me.z, ws, -wz);
                gx += __shfl_xor(gx, 32, kWave);
                gy += __shfl_xor(gy, 32, kWave);
                gz += __shfl_xor(gz, 32, kWave);
                // W is 3/8 of the accumulated sums
                const double sc = 0.75 * double(nu);
                fx += sc * double(gx);
                fy += sc * double(gy);
                fz += sc * double(gz);
                const int cur = tile == 0 ? TX : (tile == 1 ? TY : TZ);
                const int nxt = !more ? -1 : (tile == 0 ? NX : (tile == 1 ? NY : NZ));
                if (cur != nxt) {  // the role's tile changes: its forces go to the gradient
                    const int64_t gp = base[tile] + a;
                    if (h == 0 && gp < n) {
                        atomicAdd(G64 + 3 * gp + 0, fx);
                        atomicAdd(G64 + 3 * gp + 1, fy);
                        atomicAdd(G64 + 3 * gp + 2, fz);
                    }
                    fx = fy = fz = 0.0;
                }
            }
        }
        __syncthreads();  // the next tile reuses every LDS buffer
        if (!more) break;
        id = nid;
        lin = nlin;
        TX = NX;
        TY = NY;
        TZ = NZ;
        pv = pnext;
    }
}

// Group size R = 2^r of the persistent kernel: the largest R <= 32 that still
// leaves every block of a full grid at least one group, for the gradient (the
// groups exist for its force sums) on the maps whose ids nearly all decode to
// tiles (lambda, the linear listing).  The other maps deal single ids: five in
// six bounding-box ids decode to no tile, and with groups of 32 a block's tile
// count ranged from 0 to 1.8x the mean (the launch took 2.1x the time with a
// grid of 256 * 3 * 32 blocks, whose groups kept each block to the same 32 X
// tiles).
static int at_group_lg(uint64_t G, int map, bool grad) {
    if (!grad || (map != MAP_LAMBDA && map != MAP_LINEAR)) return 0;
    int r = 0;
    while (r < 5 && (G >> (r + 1)) >= uint64_t(kAtPersistBlocks)) ++r;
    return r;
}

template <int MAP, bool GRAD>
static void go_at(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float nu, double *G64,
                  double *eslots, unsigned long long *sslots, hipStream_t s) {
    const int r = at_group_lg(g.G, MAP, GRAD);
    const uint64_t groups = (g.G + (uint64_t(1) << r) - 1) >> r;
    const uint64_t cap = uint64_t(r == 5 ? kAtPersistBlocksG32 : kAtPersistBlocks);
    const uint64_t nblk = groups < cap ? groups : cap;
    const dim3 grid(uint32_t(nblk > 0 ? nblk : 1));
    if (sslots)
        hipLaunchKernelGGL((at_kernel<MAP, GRAD, true>), grid, dim3(kTripThreads), 0, s, g, X, n, ldx, nu,
                           G64, eslots, sslots, r);
    else
        hipLaunchKernelGGL((at_kernel<MAP, GRAD, false>), grid, dim3(kTripThreads), 0, s, g, X, n, ldx, nu,
                           G64, eslots, sslots, r);
}

int launch_triplet(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float nu, bool grad,
                   double *G64, double *eslots, unsigned long long *sslots, hipStream_t s) {
    const int kid = grad ? K_TRIP_GRAD : K_TRIP_ENERGY;
    prof_begin(kid, s);
    for_each_launch(g, [&](auto M, const MapGeom &gg) {
        constexpr int MAPK = decltype(M)::value;
        if (grad) go_at<MAPK, true>(gg, X, n, ldx, nu, G64, eslots, sslots, s);
        else go_at<MAPK, false>(gg, X, n, ldx, nu, G64, eslots, sslots, s);
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
    for_each_launch(g, [&](auto M, const MapGeom &gg) { go_lj<decltype(M)::value>(gg, X, n, ldx, eps, sig2, rc2, G64, eslots, sslots, s); });
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

SMX_CHECK_READER(check_flags_triplet)

}  // namespace smx
