// Host-side internals shared by the translation units of libsmx.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "smx.h"
#include "smx_maps.h"

namespace smx {

// Per-thread error message (smx_last_error).
int fail(int code, const char *fmt, ...);
// Map a HIP error (if any) to SMX_EHIP with a message.
int check_launch(const char *what);

// Checked builds: each kernel translation unit has its own device flag word;
// these read it (and clear it when asked).  ~0u if the copy failed.
#if SMX_CHECKED
#define SMX_CHECK_READER(name)                                                                   \
    unsigned name(bool clear) {                                                                  \
        unsigned v = 0;                                                                          \
        if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_check_flags), sizeof(v)) != hipSuccess) return ~0u; \
        if (clear) {                                                                             \
            const unsigned z = 0;                                                                \
            if (hipMemcpyToSymbol(HIP_SYMBOL(g_check_flags), &z, sizeof(z)) != hipSuccess) return ~0u; \
        }                                                                                        \
        return v;                                                                                \
    }
#else
#define SMX_CHECK_READER(name) \
    unsigned name(bool) { return 0; }
#endif
unsigned check_flags_edm(bool clear);
unsigned check_flags_gram(bool clear);
unsigned check_flags_map(bool clear);
unsigned check_flags_quad(bool clear);
unsigned check_flags_tripack(bool clear);
unsigned check_flags_triplet(bool clear);
unsigned check_flags_life(bool clear);

// Kernel ids for the timing facility (match smx_profile_read).
enum KernelId {
    K_MAP2 = 0, K_MAP3 = 1, K_EDM_DIFF = 2, K_EDM_GRAM = 3, K_GRAM_PREP = 4,
    K_TRIP_ENERGY = 5, K_TRIP_GRAD = 6, K_LJ = 7, K_FINALIZE = 8, K_TRIP_PACKED = 9, K_MAP4 = 10,
    K_QUAD_WORDS = 11, K_QUAD = 12, K_TRIP_TILED = 13, K_LIFE = 14, K_DECODE = 15, K_COUNT = 16
};
void prof_begin(int kid, hipStream_t s);
void prof_end(int kid, hipStream_t s);

// Grid for G logical blocks of `threads` threads: 1-D when it fits the 32-bit
// per-dimension thread count, else 2-D with 65536 blocks per row (a multiple
// of 8, so the XCD of a block stays blockIdx.x mod 8).  Kernels recompute the
// logical index with launch_index() and drop indices >= G.
inline dim3 grid_for(uint64_t G, int threads) {
    if (G * uint64_t(threads) < (uint64_t(1) << 32)) return dim3(uint32_t(G), 1, 1);
    const uint64_t gx = 65536;
    return dim3(uint32_t(gx), uint32_t((G + gx - 1) / gx), 1);
}

// Call f(std::integral_constant<int, MAP>{}) for the runtime map kind, so each
// launcher instantiates its kernel once per map.
template <typename F>
inline void map_switch(int map, F &&f) {
    switch (map) {
    case MAP_LAMBDA: f(std::integral_constant<int, MAP_LAMBDA>{}); break;
    case MAP_BBOX: f(std::integral_constant<int, MAP_BBOX>{}); break;
    case MAP_LINEAR: f(std::integral_constant<int, MAP_LINEAR>{}); break;
    case MAP_REC: f(std::integral_constant<int, MAP_REC>{}); break;
    case MAP_CUBE: f(std::integral_constant<int, MAP_CUBE>{}); break;
    default: f(std::integral_constant<int, MAP_BELOW>{}); break;
    }
}

// The sub-orthotopes of the recursive set in depth-first order, one launch
// each: the cube of side 2^(lg-1) at corner origin p, then the m sub-maps of
// side 2^(lg-1) at p + 2^(lg-1) e_d; a side-1 simplex is one block.  c.off
// advances by the blocks of each launch.
template <typename F>
inline void rec_launches(MapGeom &c, int lg, int32_t p0, int32_t p1, int32_t p2, int32_t p3, F &f) {
    const int h = lg > 0 ? lg - 1 : 0;
    c.c0 = p0;
    c.c1 = p1;
    c.c2 = p2;
    c.c3 = p3;
    c.lg = h;
    c.G = uint64_t(1) << (c.dim * h);
    f(std::integral_constant<int, MAP_CUBE>{}, static_cast<const MapGeom &>(c));
    c.off += c.G;
    if (lg == 0) return;
    const int32_t s = int32_t(1) << h;
    rec_launches(c, h, p0 + s, p1, p2, p3, f);
    rec_launches(c, h, p0, p1 + s, p2, p3, f);
    if (c.dim >= 3) rec_launches(c, h, p0, p1, p2 + s, p3, f);
    if (c.dim >= 4) rec_launches(c, h, p0, p1, p2, p3 + s, f);
}

// Call f(std::integral_constant<int, MAP>{}, geom) for every launch that the
// map needs: once for a single-launch map, once per sub-orthotope (MAP_CUBE)
// for MAP_REC_LAUNCH.
template <typename F>
inline void for_each_launch(const MapGeom &g, F &&f) {
    if (g.map == MAP_REC_LAUNCH) {
        MapGeom c = g;
        c.map = MAP_CUBE;
        c.off = 0;
        rec_launches(c, g.lg, 0, 0, 0, 0, f);
        return;
    }
    map_switch(int(g.map), [&](auto M) { f(M, g); });
}

// Map geometry for m-dimensional work with nb tiles per dimension.
// Returns false (with an error set) when the grid does not fit the index types.
bool make_geom(int m, int64_t nb, int map, MapGeom &g);

// ------------------------------------------------------------------ launchers
// Each returns SMX_OK or an error code; arguments are already validated.
int launch_fill_u64(uint64_t *p, size_t count, hipStream_t s);
int launch_stats_finalize(const unsigned long long *slots, uint64_t launched, int64_t *d_stats,
                          hipStream_t s);

int launch_map2(const MapGeom &g, int64_t n, int rho, int map, int strict, int32_t *tiles,
                unsigned long long *slots, hipStream_t s);
int launch_map3(const MapGeom &g, int64_t n, int rho, int map, int strict, int32_t *tiles,
                unsigned long long *slots, hipStream_t s);
int launch_map4(const MapGeom &g, int64_t n, int rho, int strict, int32_t *tiles,
                unsigned long long *slots, hipStream_t s);
int launch_decode(int m, const MapGeom &g, unsigned long long *slots, hipStream_t s);
int launch_count(int m, const MapGeom &g, int64_t n, int rho, int map, int strict,
                 unsigned long long *slots, hipStream_t s);

// FP32 difference form: 128 x 128 tiles (8 x 8 per thread) once there are
// enough of them to fill the chip, 64 x 64 (4 x 4 per thread) below that.
inline int edm_diff_tile(int64_t n) { return n >= 8192 ? 128 : 64; }
constexpr int kGramTile = 128;   // Gram form: 128 x 128 elements per block
constexpr int kEdmTiledTile = 128;  // tile edge of the tile-contiguous EDM layout (every precision)
inline int gram_tile(int64_t) { return kGramTile; }
constexpr int kGramK = 32;       // Gram K padding
// rows of the fragment-ordered BF16 operands (zero padded to a 32-row block)
__host__ __device__ inline int64_t gram_rows(int64_t n) { return (n + 31) / 32 * 32; }
int launch_edm_diff(const MapGeom &g, int tile, const float *X, int64_t n, int64_t d, int64_t ldx, float *D,
                    unsigned long long *slots, bool tiled, hipStream_t s);
int launch_gram_prep(const float *X, int64_t n, int64_t d, int64_t ldx, int64_t dpad, uint16_t *hi,
                     uint16_t *lo, float *norms, bool split, hipStream_t s);
int launch_edm_gram(const MapGeom &g, int tile, const uint16_t *hi, const uint16_t *lo, const float *norms,
                    int64_t n, int64_t dpad, bool split, float *D, unsigned long long *slots, bool tiled,
                    hipStream_t s);

constexpr int kTripTile = 32;    // Axilrod-Teller: 32^3 triplets per block
constexpr int kLjTile = 64;      // Lennard-Jones: 64 x 64 pairs per block
int launch_triplet(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float nu, bool grad,
                   double *G64, double *eslots, unsigned long long *sslots, hipStream_t s);
int launch_lj(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float eps, float sigma,
              float rc2, double *G64, double *eslots, unsigned long long *sslots, hipStream_t s);
int launch_energy_finalize(const double *eslots, double *E, hipStream_t s);
int launch_triplet_packed(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float nu, float *E,
                          unsigned long long *sslots, bool tiled, hipStream_t s);
constexpr int kQuadTile = 64;    // 4-point contacts: 64 elements per tile dimension
int launch_contact_words(const MapGeom &g, const float *X, int64_t n, int64_t ldx, float rc2, uint64_t *W,
                         int64_t npad, hipStream_t s);
int launch_quad(const MapGeom &g, const uint64_t *W, int64_t npad, int64_t n, unsigned long long *cslots,
                unsigned long long *sslots, hipStream_t s);
constexpr int kLifeTile = 64;    // cellular automaton: 64 x 64 cells per tile
int launch_life(const MapGeom &g, const uint8_t *S, uint8_t *D, int64_t n, unsigned long long *slots,
                hipStream_t s);
int launch_count_finalize(const unsigned long long *slots, int64_t *out, hipStream_t s);
int launch_valu_probe(float *out, int64_t blocks, int iters, hipStream_t s);
int launch_grad_finalize(const double *G64, int64_t n, const double *gradE, float *out,
                         hipStream_t s);
int launch_scale_grad(const float *G, int64_t n, const double *gradE, float *out, hipStream_t s);

}  // namespace smx
