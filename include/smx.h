/*
 * smx.h -- C ABI of libsmx, recursive block-space maps onto discrete
 * orthogonal simplices and the data-parallel work they drive, for AMD
 * Instinct MI355X (gfx950).
 *
 * Paper: C. A. Navarro, B. Bustos, N. Hitschfeld, "Possibilities of Recursive
 * GPU Mapping for Discrete Orthogonal Simplices" (arXiv:1610.07394).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers named d_* are device pointers (HIP device memory of the current
 *   device); everything else is host memory.  The caller owns and allocates
 *   every buffer, outputs and workspaces included: the library never
 *   allocates, frees or synchronises.  Work is enqueued on `stream` (a
 *   hipStream_t; NULL = the default stream) and is asynchronous.
 * - Return value: an smx_status.  Arguments are validated on the host before
 *   any HIP call; on failure nothing is enqueued and smx_last_error() holds a
 *   message (per host thread).  SMX_EHIP reports a failed launch; faults inside
 *   a kernel surface at the caller's next synchronisation.
 * - Simplex elements.  Pairs: 0 <= i <= j < n ("le") or i < j ("lt").
 *   Triplets: i <= j <= k < n ("le") or i < j < k ("lt").  The paper's
 *   eq. (1) bounds the coordinate sum by n, but its volume, eq. (2), counts
 *   the sum <= n-1 form; this library uses the equivalent pairs / triplets form,
 *   with V = n(n+1)/2 and n(n+1)(n+2)/6 elements (Sec. I, eq. (2)).
 * - Tiles.  Work is mapped per block: a block owns a tile of rho^m elements,
 *   tile (X, Y[, Z]) holding elements (X rho + a, Y rho + b[, Z rho + c]).
 *   nb = ceil(n / rho) tiles per dimension.  Tile targets are
 *   T2 = {X <= Y < nb} and T3 = {X <= Y <= Z < nb}.
 * - Maps (smx_map), i.e. how a launched block finds its tile:
 *     SMX_MAP_LAMBDA  the O(1) recursive block-space map lambda (Sec. III-A for
 *                     m = 2, Sec. III-C for m = 3).  Non-power-of-two nb uses
 *                     the paper's "approach n from above" (Sec. III-A): the
 *                     grid for the next power of two, blocks past nb filtered.
 *     SMX_MAP_BBOX    bounding box: identity over an nb^m grid, blocks outside
 *                     the simplex exit (Sec. I).
 *     SMX_MAP_LINEAR  linear enumeration g: Z^1 -> Z^m (Sec. I): FP32 square /
 *                     cube root of the block index plus an exact integer fix-up.
 *     SMX_MAP_LAMBDA_BELOW  the paper's "approach n from below" (Sec. III-A):
 *                     nb split into its binary digits (largest first); per
 *                     segment of m tiles, lambda over m (a power of two) for
 *                     its diagonal part and the identity for the rest --
 *                     2-simplex: the rectangle above the segment; 3-simplex:
 *                     lambda2(m) x identity and identity x (2-simplex from
 *                     below).  No filtered blocks in 2-D; in 3-D only those of
 *                     the lambda3 parts.  Block order: segment by segment, each
 *                     part in that order.
 *     SMX_MAP_RECURSIVE  the O(log n) recursive map of Sec. III-B, one launch:
 *                     the recursive orthotope set in the paper's corner
 *                     coordinates p (sum of p <= nb' - 1) -- the cube of side
 *                     s/2 at the origin, then m sub-maps of side s/2 at
 *                     (s/2) e_d, recursively, down to single blocks -- with
 *                     corner point p mapped to tile (p1, p1+p2[, p1+p2+p3]).
 *                     Blocks in depth-first order; V = nb'(nb'+1)/2 blocks for
 *                     m = 2 (none filtered) and (nb'^3 + 4 * 3^log2(nb')) / 5
 *                     for m = 3 (1/5 extra in the limit).  Each block walks
 *                     log2(nb') levels to find its tile.
 *     SMX_MAP_RECURSIVE_LAUNCH  the same set and block order with one kernel
 *                     launch per sub-orthotope (the recursive map calls the
 *                     paper argues against): (3^(log2 nb' + 1) - 1) / 2
 *                     launches for m = 3, 2 nb' - 1 for m = 2, all on `stream`
 *                     in depth-first order.
 *   The map changes only the schedule.  EDM outputs are bit-identical across
 *   maps; energies and gradients agree to rounding (atomic order).
 * - Statistics (d_stats, nullable): int64[4] =
 *     [0] elements visited, [1] checksum (wrapping uint64 sum of SplitMix64 of
 *     each element's id), [2] blocks that mapped to a tile, [3] blocks launched.
 *   Element ids: pairs le: i*n - i(i-1)/2 + (j-i) (the packed index);
 *   pairs lt: j(j-1)/2 + i; triplets le: k(k+1)(k+2)/6 + j(j+1)/2 + i;
 *   triplets lt: k(k-1)(k-2)/6 + j(j-1)/2 + i.  Each is a bijection onto
 *   [0, V).  Requesting statistics selects a slower counting kernel.
 */
#ifndef SMX_H
#define SMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SMX_OK = 0,
    SMX_EINVAL = 1,      /* bad argument (null pointer, negative size, bad enum, ...) */
    SMX_EOVERFLOW = 2,   /* a size does not fit the index types */
    SMX_EUNSUPPORTED = 3,/* valid request the library does not implement */
    SMX_EHIP = 4         /* a HIP call or kernel launch failed */
} smx_status;

typedef enum {
    SMX_MAP_LAMBDA = 0,
    SMX_MAP_BBOX = 1,
    SMX_MAP_LINEAR = 2,
    SMX_MAP_LAMBDA_BELOW = 3,
    SMX_MAP_RECURSIVE = 4,
    SMX_MAP_RECURSIVE_LAUNCH = 5
} smx_map;

typedef enum {
    SMX_EDM_FP32_DIFF = 0,      /* sum_k (x_ik - x_jk)^2 in FP32 on the vector ALUs */
    SMX_EDM_BF16_GRAM = 1,      /* |x_i|^2 + |x_j|^2 - 2 G_ij, G on BF16 MFMA, FP32 accumulation */
    SMX_EDM_SPLITBF16_GRAM = 2  /* as 1 with G = hi.hi + hi.lo + lo.hi (split BF16) */
} smx_edm_prec;

/* Interaction potential for the triplet calls. */
typedef struct {
    double nu;        /* Axilrod-Teller coefficient */
    int32_t at_on;    /* 1: include the Axilrod-Teller triplet energy */
    int32_t lj_on;    /* 1: include Lennard-Jones pairs */
    double lj_eps, lj_sigma, lj_rc; /* LJ epsilon, sigma, cutoff radius (> 0) */
} smx_pot;

/* Library version string. */
const char *smx_version(void);

/* Message of the last failed call on this host thread ("" if none). */
const char *smx_last_error(void);

/* Number of simplex elements: C(n+m-1, m) (paper eq. (2)) or C(n, m) when
 * strict != 0, for m in {2, 3, 4}.  Host only.  -1 on bad arguments or overflow. */
int64_t smx_volume(int m, int64_t n, int strict);

/* Number of blocks the map launches for n elements per dimension and tile
 * edge rho (the |Pi| of the paper, in blocks), m in {2, 3, 4}.  For
 * SMX_MAP_LAMBDA and m = 3 this is |Pi3| plus the lambda2 grid of the plane
 * Y = Z; for m = 4, the (nb'^4 - nb')/14 orthotope blocks plus the lambda3
 * grid of the plane X3 = X4.  It sizes the tile dump of smx_simplex_map2/3/4.
 * Host only; -1 on bad arguments or overflow. */
int64_t smx_parallel_blocks(int m, int64_t n, int rho, int map);

/* The same count under the name of the paper's quantity: the volume |Pi| of
 * the parallel space (Sec. I and III-A), in blocks.  Identical arguments,
 * result and errors as smx_parallel_blocks.  Host only. */
int64_t smx_parallel_volume(int m, int64_t n, int rho, int map);

/* The tiles of launched blocks first .. first+count-1, written to host memory
 * tiles[count][m] in block order (-1 for a filtered block); the range must lie
 * in [0, smx_parallel_blocks(m, n, rho, map)).  Evaluated on the host by the
 * same inline map code the kernels use, for inspection and testing; no device
 * work.  Host only. */
int smx_map_tiles_host(int m, int64_t n, int rho, int map, int64_t first, int64_t count,
                       int32_t *tiles);

/* Inverse maps: for each of `count` tiles (host int32[count][m], each in the
 * target simplex T2 / T3 of nb = ceil(n / rho) tiles), the index of the block
 * that `map` sends to it, written to host ids[count].  A tile X < Y of lambda2
 * lies on the level b = 2^L of the recursion with L = msb(X xor Y) and in its
 * square X >> (L+1) (Sec. III-A); a tile X <= Y < Z of lambda3 on the level of
 * msb(X xor Z) (the Sec. III-C reading).  Maps: LAMBDA, BBOX, LINEAR for m = 2
 * and 3 (SMX_EUNSUPPORTED otherwise); SMX_EINVAL for a tile outside the
 * simplex.  Host only. */
int smx_map_blocks_host(int m, int64_t n, int rho, int map, const int32_t *tiles, int64_t count, int64_t *ids);

/* Workspace bytes the calls below need (0 if none).  `op`: 0 = simplex_map
 * (any m), 1 = edm_packed, 2 = triplet calls, 3 = quad_contacts.  Host only;
 * 0 also on bad arguments. */
size_t smx_workspace_bytes(int op, int64_t n, int64_t d, int prec, int map);

/* Map dump over the 2-simplex (Sec. III-A).  Launches the parallel space of
 * `map` for n elements per dimension and tile edge rho (a power of two in
 * [1, 1024]); each block evaluates its map once and then visits the elements
 * of its tile (pairs le, or lt when strict != 0), counting them into d_stats.
 *   d_tiles  int32[smx_parallel_blocks(2, n, rho, map)][2] or NULL: tile (X, Y)
 *            of each launched block, in block order (x fastest), or (-1, -1)
 *            if the block is filtered.  Block order for LAMBDA: the
 *            (nb'/2) x (nb'+1) grid, nb' = next power of two >= nb; BBOX: nb x nb;
 *            LINEAR: one block per tile of T2.
 *   d_stats  int64[4] or NULL (see above).
 *   d_ws     smx_workspace_bytes(0, ...) bytes (required when d_stats != NULL).
 * n = 0 enqueues nothing and leaves the outputs untouched. */
int smx_simplex_map2(int64_t n, int rho, int map, int strict, int32_t *d_tiles,
                     int64_t *d_stats, void *d_ws, size_t ws_bytes, void *stream);

/* Map dump over the 3-simplex (Sec. III-C), as smx_simplex_map2 with
 * triplets; rho a power of two in [1, 64].  d_tiles is
 * int32[smx_parallel_blocks(3, n, rho, map)][3].  LAMBDA block order: the
 * (nb'/2) x (nb'/2) x (nb'/2 + nb'/4) orthotope Pi3 (x fastest), then the
 * lambda2 grid over nb whose tile (X, Y) is mapped to (X, Y, Y). */
int smx_simplex_map3(int64_t n, int rho, int map, int strict, int32_t *d_tiles,
                     int64_t *d_stats, void *d_ws, size_t ws_bytes, void *stream);

/* Map dump over the 4-simplex (Sec. III-D), as smx_simplex_map2 with
 * quadruplets i <= j <= k <= l (or i < j < k < l when strict != 0), element id
 * l(l+1)(l+2)(l+3)/24 + k(k+1)(k+2)/6 + j(j+1)/2 + i (strict: l(l-1)(l-2)(l-3)/24
 * + k(k-1)(k-2)/6 + j(j-1)/2 + i); rho a power of two in [1, 16].  d_tiles is
 * int32[smx_parallel_blocks(4, n, rho, map)][4], tiles X1 <= X2 <= X3 <= X4.
 * Maps: LAMBDA is the 4-simplex map built on the paper's r = 1/2, beta = 2
 * recursive set (the paper gives the set and its volume (n^4 - n)/14, not a
 * map): T4 splits into T4s = {X1 <= X2 <= X3 < X4} and the plane X3 = X4.  A
 * node of the binary recursion on [0, nb') (offset o, halves L and H of side b)
 * owns one b^4 orthotope of blocks whose leading blocks list its cross region
 * -- {X1<=X2<=X3 in L, X4 in H}, {X1<=X2 in L, X3<X4 in H}, {X1 in L,
 * X2<=X3<X4 in H}, b^2(b+1)(7b-1)/12 tiles, by exact-root unranking -- and
 * whose other blocks are filtered (5/7 extra in the limit, as the paper
 * states).  Block order: levels (b = nb'/2, nb'/4, ...), nodes by offset, then
 * a lambda3 grid over nb whose tile (X, Y, Z) becomes (X, Y, Z, Z).  BBOX is
 * an nb^4 1-D grid decoded with divisions (there is no 4-D hardware grid);
 * LINEAR lists T4 by X4, X3, X2, X1 (FP32 fourth root plus exact fix-up);
 * RECURSIVE / RECURSIVE_LAUNCH are the corner-coordinate recursion with four
 * branches.  LAMBDA_BELOW is not defined for m = 4 (SMX_EUNSUPPORTED). */
int smx_simplex_map4(int64_t n, int rho, int map, int strict, int32_t *d_tiles,
                     int64_t *d_stats, void *d_ws, size_t ws_bytes, void *stream);

/* The map alone, one lane per logical block id (Sec. III: the cost of evaluating
 * a map): every thread decodes 16 ids of the parallel space of map `map` over
 * the m-simplex of nb x ... x nb tiles (no element work, no block per tile), so
 * the time is the map's arithmetic per id plus the ids a map wastes, free of
 * block dispatch.  m = 2, 3 or 4; nb >= 0 (0: no work); LAMBDA_BELOW is not
 * defined for m = 4 (SMX_EUNSUPPORTED).
 *   d_stats  int64[4] device, required: [0] mapped ids (|T_m| = C(nb+m-1, m) for
 *            every map), [1] wrapping sum of SplitMix64 of the mapped tiles'
 *            colex ranks (X + C(Y+1, 2) + C(Z+2, 3) + C(W+3, 4), so the sum over
 *            a bijection onto T_m is that of the range [0, |T_m|)), [2] hardware
 *            blocks that mapped an id, [3] logical ids decoded (|Pi|).
 *   d_ws     >= smx_workspace_bytes(0, ...) bytes of device memory (the slots).
 * Asynchronous on `stream`. */
int smx_simplex_decode(int m, int64_t nb, int map, int64_t *d_stats, void *d_ws, size_t ws_bytes, void *stream);

/* Parallel space only (paper Sec. I and III: the cost of a map is the map plus
 * the blocks it launches).  Launches the parallel space of `map` for m in
 * {2, 3, 4}, n elements per dimension and tile edge rho (power of two, <= 1024
 * for m = 2, <= 64 for m = 3, <= 16 for m = 4) with 256-thread blocks; each block that maps to
 * a tile adds the number of simplex elements of that tile (le, or lt when
 * strict != 0), obtained in closed form, and filtered blocks exit at once.
 *   d_stats  int64[4]: [0] elements (= smx_volume(m, n, strict)), [1] 0,
 *            [2] blocks that mapped to a tile, [3] blocks launched.
 *   d_ws     smx_workspace_bytes(0, ...) bytes.
 * n = 0 writes zeros. */
int smx_simplex_count(int m, int64_t n, int rho, int map, int strict, int64_t *d_stats, void *d_ws,
                      size_t ws_bytes, void *stream);

/* Packed Euclidean distance matrix (paper Sec. I and II: the EDM is a
 * 2-simplex problem whose upper triangle suffices).
 *   d_X   FP32 [n][ldx] row-major, ldx >= d; read only.
 *   d_D   FP32 [n(n+1)/2]: D[p(i,j)] = |x_i - x_j|^2 for i <= j,
 *         p(i,j) = i n - i(i-1)/2 + (j - i) (row-major upper triangle with the
 *         diagonal).  Diagonal entries are exactly 0.
 *   prec  smx_edm_prec.  Gram variants round X to BF16 with round-to-nearest-even
 *         (hi = bf16(x), lo = bf16(x - hi)), accumulate in FP32, add FP32 norms
 *         |x|^2, clamp the result at 0.
 *   d_ws  smx_workspace_bytes(1, n, d, prec, map) bytes, or NULL when that is 0:
 *         statistics slots and, for the Gram variants, FP32 norms and the BF16
 *         hi (and lo) copies of X, rows padded to a multiple of 32 and columns
 *         to a multiple of 32, stored in the matrix-core operand order (1 KB
 *         per 32-row x 16-column block).  Its contents are scratch.
 *   d_stats nullable; counts pairs le. */
int smx_edm_packed(const float *d_X, int64_t n, int64_t d, int64_t ldx, int map, int prec,
                   float *d_D, void *d_ws, size_t ws_bytes, int64_t *d_stats, void *stream);

/* Diagnostic of the store ceiling (the path's output is smx_edm_packed's): it
 * separates the cost of the packed layout from the kernel's.
 * The same squared distances in a tile-contiguous layout: 128 x 128 tiles for
 * every precision, nb = ceil(n / 128), d_D of nb(nb+1)/2 * 16384 floats; tile
 * (X, Y), X <= Y < nb, starts at (Y(Y+1)/2 + X) * 16384 and element (i, j) sits at
 * 128 (i mod 128) + (j mod 128) of tile (i/128, j/128); entries of a tile that
 * are not pairs i <= j < n are 0.  Each tile is one contiguous 64 KB run, so
 * the stores stream.  Values are those of smx_edm_packed with the same `prec`,
 * bit for bit.  Arguments, workspace and errors as smx_edm_packed. */
int smx_edm_tiled(const float *d_X, int64_t n, int64_t d, int64_t ldx, int map, int prec, float *d_D,
                  void *d_ws, size_t ws_bytes, int64_t *d_stats, void *stream);

/* Triplet + pair interaction energy on the 3-simplex (Sec. I: the
 * triple-interaction n-body problem) and the 2-simplex (pair n-body).
 *   E = nu sum_{i<j<k} (1 + 3 cos g_i cos g_j cos g_k) / (r_ij r_jk r_ik)^3     (at_on)
 *     + sum_{i<j, r_ij < rc} 4 eps ((sigma/r)^12 - (sigma/r)^6)                 (lj_on)
 * with open boundaries and an unshifted LJ cutoff; whether a pair is inside
 * the cutoff is decided on s = fl(fma(dz,dz, fma(dy,dy, dx*dx))), d* = fl(x_j* - x_i*),
 * against fl(rc*rc).  Coincident particles give inf/NaN (not checked).
 *   d_X   FP32 [n][ldx], ldx >= 3 (only x, y, z are read).
 *   d_E   FP64 [3]: total, Axilrod-Teller part, Lennard-Jones part.
 *   d_ws  smx_workspace_bytes(2, n, 3, 0, map) bytes.
 *   d_stats nullable, int64[8]: [0..3] triplets lt, [4..7] pairs lt.
 * E = 0 for n < 3 (AT) and n < 2 (LJ). */
int smx_triplet_energy(const float *d_X, int64_t n, int64_t ldx, const smx_pot *pot, int map,
                       double *d_E, void *d_ws, size_t ws_bytes, int64_t *d_stats, void *stream);

/* Energy and its gradient in one pass: d_E as above (nullable) and
 * d_G FP32 [n][3] = dE/dx (forces are -d_G).  Per-pair derivatives are reduced
 * per block and accumulated into an FP64 gradient in the workspace. */
int smx_triplet_energy_grad(const float *d_X, int64_t n, int64_t ldx, const smx_pot *pot,
                            int map, double *d_E, float *d_G, void *d_ws, size_t ws_bytes,
                            void *stream);

/* Backward of smx_triplet_energy: d_dX FP32 [n][3] = gradE[0] * dE/dx, where
 * d_gradE is an FP64 device scalar (the incoming gradient of E). */
int smx_triplet_energy_backward(const float *d_X, int64_t n, int64_t ldx, const smx_pot *pot,
                                int map, const double *d_gradE, float *d_dX, void *d_ws,
                                size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as smx_triplet_energy_grad, with its workspace (energy slots and
 * the FP64 gradient accumulator) taken from a static device array of the
 * library instead of d_ws.  The array holds SMX_NOALLOC_MAX_N particles'
 * worth (1.6 MB); each GPU the library runs on keeps its own copy until the
 * process ends.  The call allocates nothing: no hipMalloc, hipFree or
 * allocating library routine; the array's device address is looked up once
 * per device, on the first call with that device current.
 *   d_X, n, ldx, pot, map, d_E (nullable), d_G  as smx_triplet_energy_grad.
 * n > SMX_NOALLOC_MAX_N returns SMX_EINVAL (use smx_triplet_energy_grad).
 * Every call on one GPU shares that GPU's array and clears what must start at
 * zero itself; calls that overlap on one GPU (different streams or threads
 * without ordering between them) race on it and give wrong results. */
#define SMX_NOALLOC_MAX_N 65536
int smx_triplet_energy_grad_noalloc(const float *d_X, int64_t n, int64_t ldx, const smx_pot *pot, int map,
                                    double *d_E, float *d_G, void *stream);

/* Packed per-triplet Axilrod-Teller energies (Sec. I: a 3-simplex problem
 * whose output, like the packed EDM of a 2-simplex, is one value per simplex
 * element; it needs no reduction, so it is bound by the stores).
 *   d_X   FP32 [n][ldx], ldx >= 3; read only.
 *   d_E   FP32 [n(n-1)(n-2)/6]: E[p(i,j,k)] = nu (1 + 3 cos g_i cos g_j cos g_k)
 *         / (r_ij r_jk r_ik)^3 for every i < j < k < n, p the lexicographic rank
 *         p(i,j,k) = C(n,3) - C(n-i,3) + (j-i-1)(n-1) - (j(j-1)/2 - i(i+1)/2)
 *                    + (k-j-1).  FP32 arithmetic in the kernel.
 *   map   smx_map (lambda3 over 32^3 tiles, or a baseline); the result does not
 *         depend on it.
 *   d_stats nullable; with d_ws of smx_workspace_bytes(0, n) bytes it counts
 *         the stored elements (triplets lt) and their checksum.
 * n <= 2^21 (SMX_EOVERFLOW beyond); n < 3 writes nothing. */
int smx_triplet_packed(const float *d_X, int64_t n, int64_t ldx, double nu, int map, float *d_E, void *d_ws,
                       size_t ws_bytes, int64_t *d_stats, void *stream);

/* Diagnostic of the store ceiling (the path's output is smx_triplet_packed's):
 * it separates the cost of the packed layout from the kernel's.
 * The same per-triplet energies in a tile-contiguous layout, so that each
 * 32^3 tile is written as one contiguous 128 KB run.  With nb = ceil(n / 32),
 * d_E holds C(nb+2, 3) * 32768 floats: tile (X, Y, Z), X <= Y <= Z < nb, starts
 * at rank * 32768 with rank = Z(Z+1)(Z+2)/6 + Y(Y+1)/2 + X, and triplet (i, j, k)
 * sits at offset 1024 (i mod 32) + 32 (j mod 32) + (k mod 32) of tile
 * (i/32, j/32, k/32); the entries of a tile that are not triplets i < j < k < n
 * are 0.  The values are those of smx_triplet_packed, bit for bit.  Arguments,
 * limits and errors as smx_triplet_packed. */
int smx_triplet_packed_tiled(const float *d_X, int64_t n, int64_t ldx, double nu, int map, float *d_E,
                             void *d_ws, size_t ws_bytes, int64_t *d_stats, void *stream);

/* 4-point contacts on the 4-simplex (Sec. I: correlation counts over the
 * simplex; Sec. III-D: the 4-simplex parallel space).  Counts the quadruplets
 * i < j < k < l whose six pairs are all in contact -- the 4-cliques of the
 * contact graph -- where a pair i < j is in contact when the FP32 squared
 * distance fl(fma(dz,dz, fma(dy,dy, dx*dx))), d* = fl(x_j* - x_i*), is below
 * fl(rc*rc).  Two passes over 64-element tiles: contact bit words over the
 * 2-simplex (map `map` with m = 2), then the cliques over the 4-simplex (map
 * `map` with m = 4; LAMBDA is the lambda4 map of smx_simplex_map4).
 *   d_X      FP32 [n][ldx] device, x, y, z in columns 0..2; ldx >= 3.
 *   n        0 <= n <= 16384 (n < 4 gives 0).
 *   rc       contact radius, finite and >= 0.
 *   map      smx_map; LAMBDA_BELOW is not defined for m = 4 (SMX_EUNSUPPORTED).
 *   d_count  int64[1] device: the number of 4-cliques (exact).
 *   d_ws     smx_workspace_bytes(3, n, 3, 0, map) bytes of device memory:
 *            count and statistics slots, then the contact words, 64-bit,
 *            column-tile-major: word [Y][64 X + p] holds the contacts of row
 *            64 X + p with columns 64 Y .. 64 Y + 63 (upper tiles X <= Y only).
 *   d_stats  int64[4] or NULL: [0] quadruplets covered (C(n, 4) when every tile
 *            is visited once), [1] 0, [2] mapped 4-simplex blocks, [3] 4-simplex
 *            blocks of the parallel space (logical blocks: the clique pass
 *            decodes them one per lane, 256 per hardware block).
 * Asynchronous on `stream`; the result is exact, so every map returns the same
 * count. */
int smx_quad_contacts(const float *d_X, int64_t n, int64_t ldx, double rc, int map, int64_t *d_count,
                      void *d_ws, size_t ws_bytes, int64_t *d_stats, void *stream);

/* Measurement probe for the roofline of the VALU-bound kernels (not part of
 * the simplex path): enqueues `blocks` blocks of 256 threads, each thread
 * running iters x 64 FP32 fused multiply-adds in eight independent chains with
 * no memory traffic, then one store to d_out[blocks * 256] (FP32, device,
 * caller-owned).  The caller times it on `stream`; lane operations =
 * blocks * 256 * iters * 64.  blocks in [1, 2^24], iters >= 1. */
int smx_probe_valu(float *d_out, int64_t blocks, int iters, void *stream);

/* Device checks.  The library can be built a second time with SMX_CHECKED=1
 * (libsmx_checked.so, same ABI): every map evaluation then verifies that its
 * tile lies in the simplex, and every unmasked store on a tile taken for
 * interior verifies that its element does; a violation skips the access and
 * sets a flag bit (1: a map left the simplex, 2: a store left it).  Callers
 * that want a map or a kernel checked run it through that library and read
 * the flags here, which synchronises with the device.
 *   flags  host uint32 out: the OR of the flags of all kernels.
 *   clear  != 0: reset the flags after reading them.
 * SMX_EUNSUPPORTED in the normal library (no checks compiled in). */
int smx_check_flags(uint32_t *flags, int clear);

/* One generation of Conway's Life on the 2-simplex of cells (i, j), 0 <= i <=
 * j < n: a cellular automaton on a triangular domain (Sec. I).  Birth on 3 live
 * neighbours, survival on 2 or 3 (Moore neighbourhood); cells outside the
 * triangle are dead.  Tiles of 64 x 64 cells on the 2-simplex map `map`.
 *   d_in, d_out  uint8 device buffers of nb(nb+1)/2 * 4096 bytes, nb = ceil(n/64),
 *                tile-contiguous: tile (X, Y), X <= Y < nb, at (Y(Y+1)/2 + X) * 4096,
 *                cell (i, j) at 64 (i mod 64) + (j mod 64), 1 = alive.  d_out gets 0
 *                outside the triangle; d_in is not read there.  Distinct buffers
 *                (a caller stepping several generations alternates them).
 *   d_stats      int64[4] or NULL: [0] live cells after the step, [1] 0, [2] mapped
 *                blocks, [3] launched blocks (d_ws of smx_workspace_bytes(0, ...)).
 * n <= 2^24. */
int smx_simplex_life(const uint8_t *d_in, uint8_t *d_out, int64_t n, int map, int64_t *d_stats, void *d_ws,
                     size_t ws_bytes, void *stream);

/* d_out[q] = gradE[0] * d_G[q] for q < 3n (FP32 out, FP64 scale): the backward
 * pass of smx_triplet_energy_grad's output, given the incoming gradient
 * d_gradE (FP64 device scalar).  d_out may alias d_G. */
int smx_scale_grad(const float *d_G, int64_t n, const double *d_gradE, float *d_out, void *stream);

/* Kernel timing: when enabled, every main kernel launch is bracketed by HIP
 * events on its own stream.  smx_profile_read synchronises on those events and
 * returns the summed duration (ms) and launch count of kernel `kernel_id`
 * (0 map2, 1 map3, 2 edm diff, 3 edm gram, 4 gram prep, 5 triplet energy,
 * 6 triplet grad, 7 lj, 8 finalize, 9 triplet packed, 10 map4, 11 contact words,
 * 12 quad contacts, 13 triplet packed tiled, 14 life, 15 decode) since the last reset; it
 * returns SMX_EINVAL
 * for an unknown id.  smx_profile_reset clears the totals.  Host only. */
int smx_profile_enable(int on);
int smx_profile_reset(void);
int smx_profile_read(int kernel_id, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* SMX_H */
