// C ABI of libsmx: argument validation, workspace layout, and the sequence
// of kernel launches behind each entry point.  Everything is enqueued on the
// caller's stream; nothing here allocates device memory or synchronises
// (except the explicit timing read-out).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "smx_device.h"
#include "smx_internal.h"
#include "smx_maps_inv.h"

namespace smx {

static thread_local char g_err[512] = "";
// Code of the last fail() on this thread: what a failed make_geom reported.
static thread_local int g_status = SMX_OK;

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    g_status = code;
    return code;
}

int check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SMX_EHIP, "%s: launch failed: %s", what, hipGetErrorString(e));
    return SMX_OK;
}

// ------------------------------------------------------------------ timing
namespace {
struct Rec {
    int kid;
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_prof = false;
std::vector<Rec> g_pending;
hipEvent_t g_open[K_COUNT] = {};
double g_tot[K_COUNT] = {};
int64_t g_cnt[K_COUNT] = {};
}  // namespace

void prof_begin(int kid, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_prof) return;
    hipEvent_t a;
    if (hipEventCreate(&a) != hipSuccess) return;
    hipEventRecord(a, s);
    g_open[kid] = a;
}

void prof_end(int kid, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_prof || g_open[kid] == nullptr) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) return;
    hipEventRecord(b, s);
    g_pending.push_back({kid, g_open[kid], b});
    g_open[kid] = nullptr;
}

static void prof_collect() {
    for (const Rec &r : g_pending) {
        float ms = 0.f;
        hipEventSynchronize(r.b);
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            g_tot[r.kid] += ms;
            g_cnt[r.kid] += 1;
        }
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    g_pending.clear();
}

// ------------------------------------------------------------------ geometry
static bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

static constexpr uint64_t kMaxBlocks = (uint64_t(1) << 31) - 1;
static constexpr int64_t kMaxN = (int64_t(1) << 31) - 1;
static constexpr int64_t kMaxGridDim = 65535;

bool make_geom(int m, int64_t nb, int map, MapGeom &g) {
    memset(&g, 0, sizeof(g));
    g.nb = int32_t(nb);
    g.map = uint32_t(map);
    g.dim = m;
    const uint64_t u = uint64_t(nb);
    if (m == 4) {
        if (map == MAP_BELOW)
            return fail(SMX_EUNSUPPORTED, "the from-below map is defined for m = 2 and 3 only"), false;
        if (nb > 65535) return fail(SMX_EOVERFLOW, "grid too large (nb = %lld)", (long long)nb), false;
        if (map == MAP_LAMBDA) {
            g.lg = ceil_log2_u64(u);
            if (g.lg > 8) return fail(SMX_EOVERFLOW, "lambda4 grid too large (nb = %lld)", (long long)nb), false;
            g.main = uint32_t(lambda4_main_blocks(g.lg));
            g.G = g.main + lambda3_main_blocks(g.lg) + lambda2_blocks(g.lg);
        } else if (map == MAP_REC || map == MAP_REC_LAUNCH) {
            g.lg = ceil_log2_u64(u);
            if (g.lg > 15) return fail(SMX_EOVERFLOW, "recursive grid too large (nb = %lld)", (long long)nb), false;
            g.G = rec_blocks(4, g.lg);
        } else if (map == MAP_BBOX) {
            g.G = u * u * u * u;
        } else {
            g.G = u * (u + 1) * (u + 2) * (u + 3) / 24;
        }
    } else if (map == MAP_REC || map == MAP_REC_LAUNCH) {
        g.lg = ceil_log2_u64(u);
        if (g.lg > 20) return fail(SMX_EOVERFLOW, "recursive grid too large (nb = %lld)", (long long)nb), false;
        g.G = rec_blocks(m, g.lg);
    } else if (map == MAP_LAMBDA) {
        g.lg = ceil_log2_u64(u);
        if (g.lg > 30) return fail(SMX_EOVERFLOW, "lambda grid too large (nb = %lld)", (long long)nb), false;
        const uint64_t g2 = lambda2_blocks(g.lg);
        if (m == 2) {
            g.G = g2;
        } else {
            if (g.lg > 21) return fail(SMX_EOVERFLOW, "lambda3 grid too large (nb = %lld)", (long long)nb), false;
            const uint64_t half = g.lg == 0 ? 0 : (uint64_t(1) << (g.lg - 1));
            const uint64_t main = half * half * (half + half / 2);
            if (main > kMaxBlocks) return fail(SMX_EOVERFLOW, "lambda3 grid too large"), false;
            g.main = uint32_t(main);
            g.G = main + g2;
        }
    } else if (map == MAP_BELOW) {
        if (nb > (int64_t(1) << 24)) return fail(SMX_EOVERFLOW, "grid too large (nb = %lld)", (long long)nb), false;
        g.G = m == 2 ? below2_blocks(u) : below3_blocks(u);
    } else if (map == MAP_BBOX) {
        if (nb > kMaxGridDim) return fail(SMX_EUNSUPPORTED, "bounding-box grid dimension %lld > 65535", (long long)nb), false;
        g.G = m == 2 ? u * u : u * u * u;
    } else {
        g.G = m == 2 ? u * (u + 1) / 2 : u * (u + 1) * (u + 2) / 6;
    }
    if (g.G > kMaxBlocks) return fail(SMX_EOVERFLOW, "parallel space of %llu blocks exceeds 2^31 - 1", (unsigned long long)g.G), false;
    return true;
}

// Largest tile edge per dimension: the element-visiting kernels loop over
// rho^m elements per block.
static int max_rho(int m) { return m == 2 ? 1024 : m == 3 ? 64 : 16; }

static int check_common(int m, int64_t n, int rho, int map, int maxrho) {
    if (m < 2 || m > 4) return fail(SMX_EINVAL, "m must be 2, 3 or 4 (got %d)", m);
    if (n < 0) return fail(SMX_EINVAL, "n must be >= 0 (got %lld)", (long long)n);
    if (n > kMaxN) return fail(SMX_EOVERFLOW, "n = %lld exceeds 2^31 - 1", (long long)n);
    if (!pow2(rho) || rho > maxrho) return fail(SMX_EINVAL, "rho must be a power of two in [1, %d] (got %d)", maxrho, rho);
    if (map < 0 || map > MAP_REC_LAUNCH) return fail(SMX_EINVAL, "unknown map %d", map);
    return SMX_OK;
}

static inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Workspace layouts.
struct EdmWs {
    size_t slots, hi, lo, norms, total;
};
static EdmWs edm_ws(int64_t n, int64_t d, int prec) {
    EdmWs w{};
    w.slots = 0;
    size_t off = kSlotBytes;
    if (prec != SMX_EDM_FP32_DIFF) {
        const int64_t dpad = (d + kGramK - 1) / kGramK * kGramK;
        const int64_t npad = gram_rows(n);
        w.hi = off;
        off = align256(off + size_t(npad) * size_t(dpad) * 2);
        w.lo = off;
        if (prec == SMX_EDM_SPLITBF16_GRAM) off = align256(off + size_t(npad) * size_t(dpad) * 2);
        w.norms = off;
        off = align256(off + size_t(n) * 4);
    }
    w.total = off;
    return w;
}

struct TripWs {
    size_t eslots, at_stats, lj_stats, g64, total;
};
static TripWs trip_ws(int64_t n) {
    TripWs w{};
    w.eslots = 0;
    w.at_stats = kSlotBytes;
    w.lj_stats = 2 * kSlotBytes;
    w.g64 = 3 * kSlotBytes;
    w.total = align256(w.g64 + size_t(n) * 3 * 8);
    return w;
}

struct QuadWs {
    size_t cslots, sslots, words, total;
    int64_t nb, npad;
};
static QuadWs quad_ws(int64_t n) {
    QuadWs w{};
    w.nb = (n + kQuadTile - 1) / kQuadTile;
    w.npad = w.nb * kQuadTile;
    w.cslots = 0;
    w.sslots = kSlotBytes;
    w.words = 2 * kSlotBytes;
    w.total = align256(w.words + size_t(w.nb) * size_t(w.npad) * 8);
    return w;
}

static inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace smx

using namespace smx;

extern "C" {

const char *smx_version(void) { return "smx 0.1 (gfx950)"; }

const char *smx_last_error(void) { return g_err; }

int64_t smx_volume(int m, int64_t n, int strict) {
    if (m < 2 || m > 4 || n < 0 || n > kMaxN) return -1;
    const __int128 a = n, b = strict ? n - 1 : n + 1;
    __int128 v;
    if (m == 2) v = a * b / 2;
    else if (m == 3) v = strict ? a * (n - 1) * (n - 2) / 6 : a * (n + 1) * (n + 2) / 6;
    else v = strict ? a * (n - 1) * (n - 2) * (n - 3) / 24 : a * (n + 1) * (n + 2) * (n + 3) / 24;
    if (v < 0) v = 0;
    if (v > (__int128)INT64_MAX) return -1;
    return int64_t(v);
}

int64_t smx_parallel_blocks(int m, int64_t n, int rho, int map) {
    if (check_common(m, n, rho, map, max_rho(m)) != SMX_OK) return -1;
    if (n == 0) return 0;
    MapGeom g;
    if (!make_geom(m, (n + rho - 1) / rho, map, g)) return -1;
    return int64_t(g.G);
}

int64_t smx_parallel_volume(int m, int64_t n, int rho, int map) { return smx_parallel_blocks(m, n, rho, map); }

size_t smx_workspace_bytes(int op, int64_t n, int64_t d, int prec, int map) {
    (void)map;
    if (n < 0 || n > kMaxN) return 0;
    if (op == 0) return kSlotBytes;
    if (op == 1) {
        if (d < 1 || prec < 0 || prec > 2) return 0;
        return edm_ws(n, d, prec).total;
    }
    if (op == 2) return trip_ws(n).total;
    if (op == 3) return quad_ws(n).total;
    return 0;
}

int smx_map_tiles_host(int m, int64_t n, int rho, int map, int64_t first, int64_t count, int32_t *tiles) {
    int rc = check_common(m, n, rho, map, max_rho(m));
    if (rc != SMX_OK) return rc;
    if (count < 0 || first < 0) return fail(SMX_EINVAL, "negative block range");
    if (count == 0) return SMX_OK;
    if (tiles == nullptr) return fail(SMX_EINVAL, "tiles is NULL");
    MapGeom g;
    if (n == 0) return fail(SMX_EINVAL, "n = 0 launches no blocks");
    if (!make_geom(m, (n + rho - 1) / rho, map, g)) return g_status;
    if (uint64_t(first) + uint64_t(count) > g.G) return fail(SMX_EINVAL, "block range past the parallel space");
    for (uint64_t b = uint64_t(first); b < uint64_t(first + count); ++b) {
        int X = -1, Y = -1, Z = -1;
        int32_t *o = tiles + (b - uint64_t(first)) * m;
        bool ok;
        if (m == 4) {
            int T[4] = {-1, -1, -1, -1};
            if (map == MAP_LAMBDA) ok = lambda4(uint32_t(b), g.lg, g.nb, g.main, T);
            else if (map == MAP_BBOX) {
                uint64_t r = b;
                for (int d = 0; d < 4; ++d) {
                    T[d] = int(r % uint64_t(g.nb));
                    r /= uint64_t(g.nb);
                }
                ok = T[0] <= T[1] && T[1] <= T[2] && T[2] <= T[3];
            } else if (map == MAP_REC || map == MAP_REC_LAUNCH) ok = rec4(uint32_t(b), g.lg, g.nb, uint32_t(g.G), T);
            else { linear4(uint32_t(b), T); ok = true; }
            for (int d = 0; d < 4; ++d) o[d] = ok ? T[d] : -1;
        } else if (m == 2) {
            if (map == MAP_LAMBDA) ok = lambda2(uint32_t(b), g.lg, g.nb, X, Y);
            else if (map == MAP_BBOX) { X = int(b % g.nb); Y = int(b / g.nb); ok = X <= Y; }
            else if (map == MAP_BELOW) ok = below2(b, uint32_t(g.nb), X, Y);
            else if (map == MAP_REC || map == MAP_REC_LAUNCH) ok = rec2(uint32_t(b), g.lg, g.nb, uint32_t(g.G), X, Y);
            else { linear2(uint32_t(b), X, Y); ok = true; }
            o[0] = ok ? X : -1;
            o[1] = ok ? Y : -1;
        } else {
            if (map == MAP_LAMBDA) ok = lambda3(uint32_t(b), g.lg, g.nb, g.main, X, Y, Z);
            else if (map == MAP_BBOX) {
                X = int(b % g.nb); Y = int((b / g.nb) % g.nb); Z = int(b / (uint64_t(g.nb) * g.nb));
                ok = X <= Y && Y <= Z;
            } else if (map == MAP_BELOW) ok = below3(b, uint32_t(g.nb), X, Y, Z);
            else if (map == MAP_REC || map == MAP_REC_LAUNCH) ok = rec3(uint32_t(b), g.lg, g.nb, uint32_t(g.G), X, Y, Z);
            else { linear3(uint32_t(b), X, Y, Z); ok = true; }
            o[0] = ok ? X : -1;
            o[1] = ok ? Y : -1;
            o[2] = ok ? Z : -1;
        }
    }
    return SMX_OK;
}

int smx_map_blocks_host(int m, int64_t n, int rho, int map, const int32_t *tiles, int64_t count, int64_t *ids) {
    int rc = check_common(m, n, rho, map, max_rho(m));
    if (rc != SMX_OK) return rc;
    if (m == 4 || (map != MAP_LAMBDA && map != MAP_BBOX && map != MAP_LINEAR))
        return fail(SMX_EUNSUPPORTED, "inverse maps exist for lambda, bounding box and linear with m = 2, 3");
    if (count < 0) return fail(SMX_EINVAL, "negative count");
    if (count == 0) return SMX_OK;
    if (tiles == nullptr || ids == nullptr) return fail(SMX_EINVAL, "tiles and ids must not be NULL");
    if (n == 0) return fail(SMX_EINVAL, "n = 0 has no tiles");
    MapGeom g;
    if (!make_geom(m, (n + rho - 1) / rho, map, g)) return g_status;
    for (int64_t e = 0; e < count; ++e) {
        const int32_t *t = tiles + e * m;
        bool in = true;
        for (int d = 0; d < m; ++d) in = in && t[d] >= 0 && t[d] < g.nb && (d == 0 || t[d - 1] <= t[d]);
        if (!in) return fail(SMX_EINVAL, "tile %lld is not in the simplex", (long long)e);
        const uint32_t X = uint32_t(t[0]), Y = uint32_t(t[1]), Z = m == 3 ? uint32_t(t[2]) : 0;
        uint64_t id;
        if (map == MAP_LAMBDA) id = m == 2 ? lambda2_inv(g.lg, X, Y) : lambda3_inv(g.lg, g.main, X, Y, Z);
        else if (map == MAP_BBOX) id = m == 2 ? uint64_t(Y) * g.nb + X : (uint64_t(Z) * g.nb + Y) * g.nb + X;
        else id = m == 2 ? linear2_inv(X, Y) : linear3_inv(X, Y, Z);
        ids[e] = int64_t(id);
    }
    return SMX_OK;
}

static int map_dump(int m, int64_t n, int rho, int map, int strict, int32_t *d_tiles, int64_t *d_stats,
                    void *d_ws, size_t ws_bytes, void *stream) {
    int rc = check_common(m, n, rho, map, max_rho(m));
    if (rc != SMX_OK) return rc;
    if (d_stats != nullptr && (d_ws == nullptr || ws_bytes < kSlotBytes))
        return fail(SMX_EINVAL, "statistics need a workspace of %zu bytes", kSlotBytes);
    if (n == 0) return SMX_OK;
    MapGeom g;
    if (!make_geom(m, (n + rho - 1) / rho, map, g)) return g_status;
    unsigned long long *slots = d_stats ? reinterpret_cast<unsigned long long *>(d_ws) : nullptr;
    if (slots && (rc = launch_fill_u64(reinterpret_cast<uint64_t *>(slots), kSlotBytes / 8, S(stream))))
        return rc;
    rc = m == 2   ? launch_map2(g, n, rho, map, strict, d_tiles, slots, S(stream))
         : m == 3 ? launch_map3(g, n, rho, map, strict, d_tiles, slots, S(stream))
                  : launch_map4(g, n, rho, strict, d_tiles, slots, S(stream));
    if (rc) return rc;
    if (slots) return launch_stats_finalize(slots, g.G, d_stats, S(stream));
    return SMX_OK;
}

int smx_simplex_map2(int64_t n, int rho, int map, int strict, int32_t *d_tiles, int64_t *d_stats,
                     void *d_ws, size_t ws_bytes, void *stream) {
    return map_dump(2, n, rho, map, strict, d_tiles, d_stats, d_ws, ws_bytes, stream);
}

int smx_simplex_map3(int64_t n, int rho, int map, int strict, int32_t *d_tiles, int64_t *d_stats,
                     void *d_ws, size_t ws_bytes, void *stream) {
    return map_dump(3, n, rho, map, strict, d_tiles, d_stats, d_ws, ws_bytes, stream);
}

int smx_simplex_map4(int64_t n, int rho, int map, int strict, int32_t *d_tiles, int64_t *d_stats,
                     void *d_ws, size_t ws_bytes, void *stream) {
    return map_dump(4, n, rho, map, strict, d_tiles, d_stats, d_ws, ws_bytes, stream);
}

int smx_simplex_count(int m, int64_t n, int rho, int map, int strict, int64_t *d_stats, void *d_ws,
                      size_t ws_bytes, void *stream) {
    int rc = check_common(m, n, rho, map, max_rho(m));
    if (rc != SMX_OK) return rc;
    if (d_stats == nullptr) return fail(SMX_EINVAL, "stats must not be NULL");
    if (d_ws == nullptr || ws_bytes < kSlotBytes)
        return fail(SMX_EINVAL, "a workspace of %zu bytes is required", kSlotBytes);
    MapGeom g{};
    if (n > 0 && !make_geom(m, (n + rho - 1) / rho, map, g)) return g_status;
    unsigned long long *slots = reinterpret_cast<unsigned long long *>(d_ws);
    if ((rc = launch_fill_u64(reinterpret_cast<uint64_t *>(slots), kSlotBytes / 8, S(stream)))) return rc;
    if (n > 0 && (rc = launch_count(m, g, n, rho, map, strict, slots, S(stream)))) return rc;
    return launch_stats_finalize(slots, g.G, d_stats, S(stream));
}

int smx_simplex_decode(int m, int64_t nb, int map, int64_t *d_stats, void *d_ws, size_t ws_bytes, void *stream) {
    if (m < 2 || m > 4) return fail(SMX_EINVAL, "m must be 2, 3 or 4 (got %d)", m);
    if (nb < 0) return fail(SMX_EINVAL, "nb must be >= 0 (got %lld)", (long long)nb);
    if (nb > kMaxN) return fail(SMX_EOVERFLOW, "nb = %lld exceeds 2^31 - 1", (long long)nb);
    if (map < 0 || map > MAP_REC_LAUNCH) return fail(SMX_EINVAL, "unknown map %d", map);
    if (d_stats == nullptr) return fail(SMX_EINVAL, "stats must not be NULL");
    if (d_ws == nullptr || ws_bytes < kSlotBytes)
        return fail(SMX_EINVAL, "a workspace of %zu bytes is required", kSlotBytes);
    MapGeom g{};
    if (nb > 0 && !make_geom(m, nb, map, g)) return g_status;
    unsigned long long *slots = reinterpret_cast<unsigned long long *>(d_ws);
    int rc;
    if ((rc = launch_fill_u64(reinterpret_cast<uint64_t *>(slots), kSlotBytes / 8, S(stream)))) return rc;
    if (nb > 0 && (rc = launch_decode(m, g, slots, S(stream)))) return rc;
    return launch_stats_finalize(slots, g.G, d_stats, S(stream));
}

static int edm_run(bool tiled, const float *d_X, int64_t n, int64_t d, int64_t ldx, int map, int prec, float *d_D,
                   void *d_ws, size_t ws_bytes, int64_t *d_stats, void *stream) {
    if (n < 0) return fail(SMX_EINVAL, "n must be >= 0");
    if (n > kMaxN) return fail(SMX_EOVERFLOW, "n exceeds 2^31 - 1");
    if (d < 1) return fail(SMX_EINVAL, "d must be >= 1 (got %lld)", (long long)d);
    if (ldx < d) return fail(SMX_EINVAL, "ldx (%lld) < d (%lld)", (long long)ldx, (long long)d);
    if (map < 0 || map > MAP_REC_LAUNCH) return fail(SMX_EINVAL, "unknown map %d", map);
    if (prec < 0 || prec > 2) return fail(SMX_EINVAL, "unknown precision %d", prec);
    if (n == 0) return SMX_OK;
    if (d_X == nullptr || d_D == nullptr) return fail(SMX_EINVAL, "X and D must not be NULL");
    const EdmWs w = edm_ws(n, d, prec);
    const bool need_ws = prec != SMX_EDM_FP32_DIFF || d_stats != nullptr;
    if (need_ws && (d_ws == nullptr || ws_bytes < w.total))
        return fail(SMX_EINVAL, "workspace of %zu bytes required (got %zu)", w.total, ws_bytes);
    const int tile = tiled ? kEdmTiledTile : prec == SMX_EDM_FP32_DIFF ? edm_diff_tile(n) : gram_tile(n);
    MapGeom g;
    if (!make_geom(2, (n + tile - 1) / tile, map, g)) return g_status;
    char *ws = reinterpret_cast<char *>(d_ws);
    unsigned long long *slots = d_stats ? reinterpret_cast<unsigned long long *>(ws + w.slots) : nullptr;
    int rc;
    if (slots && (rc = launch_fill_u64(reinterpret_cast<uint64_t *>(slots), kSlotBytes / 8, S(stream))))
        return rc;
    if (prec == SMX_EDM_FP32_DIFF) {
        rc = launch_edm_diff(g, tile, d_X, n, d, ldx, d_D, slots, tiled, S(stream));
    } else {
        const bool split = prec == SMX_EDM_SPLITBF16_GRAM;
        const int64_t dpad = (d + kGramK - 1) / kGramK * kGramK;
        uint16_t *hi = reinterpret_cast<uint16_t *>(ws + w.hi);
        uint16_t *lo = reinterpret_cast<uint16_t *>(ws + w.lo);
        float *norms = reinterpret_cast<float *>(ws + w.norms);
        rc = launch_gram_prep(d_X, n, d, ldx, dpad, hi, lo, norms, split, S(stream));
        if (rc == SMX_OK) rc = launch_edm_gram(g, tile, hi, lo, norms, n, dpad, split, d_D, slots, tiled, S(stream));
    }
    if (rc) return rc;
    if (slots) return launch_stats_finalize(slots, g.G, d_stats, S(stream));
    return SMX_OK;
}

int smx_edm_packed(const float *d_X, int64_t n, int64_t d, int64_t ldx, int map, int prec, float *d_D,
                   void *d_ws, size_t ws_bytes, int64_t *d_stats, void *stream) {
    return edm_run(false, d_X, n, d, ldx, map, prec, d_D, d_ws, ws_bytes, d_stats, stream);
}

int smx_edm_tiled(const float *d_X, int64_t n, int64_t d, int64_t ldx, int map, int prec, float *d_D,
                  void *d_ws, size_t ws_bytes, int64_t *d_stats, void *stream) {
    return edm_run(true, d_X, n, d, ldx, map, prec, d_D, d_ws, ws_bytes, d_stats, stream);
}

static int check_pot(const smx_pot *pot) {
    if (pot == nullptr) return fail(SMX_EINVAL, "pot is NULL");
    if (pot->lj_on && !(pot->lj_rc > 0.0 && pot->lj_sigma > 0.0))
        return fail(SMX_EINVAL, "LJ needs sigma > 0 and rc > 0");
    return SMX_OK;
}

static void *scratch_for_current_device();

// Shared body of the triplet calls.  mode 0: energy; 1: energy + gradient;
// 2: backward (gradient scaled by *d_gradE).  static_ws: take the workspace
// from the library's static device array (after every argument check, so a
// bad call still touches no device state) instead of d_ws.
static int triplet_run(int mode, const float *d_X, int64_t n, int64_t ldx, const smx_pot *pot, int map,
                       double *d_E, float *d_G, const double *d_gradE, void *d_ws, size_t ws_bytes,
                       int64_t *d_stats, void *stream, bool static_ws = false) {
    if (n < 0) return fail(SMX_EINVAL, "n must be >= 0");
    if (n > kMaxN) return fail(SMX_EOVERFLOW, "n exceeds 2^31 - 1");
    if (ldx < 3) return fail(SMX_EINVAL, "ldx must be >= 3 (got %lld)", (long long)ldx);
    if (map < 0 || map > MAP_REC_LAUNCH) return fail(SMX_EINVAL, "unknown map %d", map);
    int rc = check_pot(pot);
    if (rc) return rc;
    if (mode == 0 && d_E == nullptr) return fail(SMX_EINVAL, "E must not be NULL");
    if (mode >= 1 && n > 0 && d_G == nullptr) return fail(SMX_EINVAL, "gradient output must not be NULL");
    if (mode == 2 && d_gradE == nullptr) return fail(SMX_EINVAL, "gradE must not be NULL");
    if (n > 0 && d_X == nullptr) return fail(SMX_EINVAL, "X must not be NULL");
    const TripWs w = trip_ws(n);
    if (!static_ws && (d_ws == nullptr || ws_bytes < w.total))
        return fail(SMX_EINVAL, "workspace of %zu bytes required (got %zu)", w.total, ws_bytes);
    MapGeom g3, g2;
    const int64_t nb3 = (n + kTripTile - 1) / kTripTile, nb2 = (n + kLjTile - 1) / kLjTile;
    const bool do_at = pot->at_on && n >= 3, do_lj = pot->lj_on && n >= 2;
    if (do_at && !make_geom(3, nb3, map, g3)) return g_status;
    if (do_lj && !make_geom(2, nb2, map, g2)) return g_status;
    if (static_ws) {
        if ((d_ws = scratch_for_current_device()) == nullptr) return g_status;
        ws_bytes = w.total;
    }

    char *ws = reinterpret_cast<char *>(d_ws);
    double *eslots = reinterpret_cast<double *>(ws + w.eslots);
    unsigned long long *at_st = d_stats ? reinterpret_cast<unsigned long long *>(ws + w.at_stats) : nullptr;
    unsigned long long *lj_st = d_stats ? reinterpret_cast<unsigned long long *>(ws + w.lj_stats) : nullptr;
    double *G64 = reinterpret_cast<double *>(ws + w.g64);
    hipStream_t s = S(stream);
    // zero energy slots, statistics slots and the FP64 gradient in one fill
    const size_t zero_words = (mode == 0 ? (d_stats ? w.g64 : w.at_stats) : w.total) / 8;
    if ((rc = launch_fill_u64(reinterpret_cast<uint64_t *>(ws), zero_words, s))) return rc;
    const bool grad = mode >= 1;
    if (do_at && (rc = launch_triplet(g3, d_X, n, ldx, float(pot->nu), grad, G64, eslots, at_st, s))) return rc;
    if (do_lj && (rc = launch_lj(g2, d_X, n, ldx, float(pot->lj_eps), float(pot->lj_sigma),
                                 float(pot->lj_rc * pot->lj_rc), G64, eslots, lj_st, s)))
        return rc;
    if (d_E != nullptr && (rc = launch_energy_finalize(eslots, d_E, s))) return rc;
    if (d_stats != nullptr) {
        if ((rc = launch_stats_finalize(at_st, do_at ? g3.G : 0, d_stats, s))) return rc;
        if ((rc = launch_stats_finalize(lj_st, do_lj ? g2.G : 0, d_stats + 4, s))) return rc;
    }
    if (grad && n > 0 && (rc = launch_grad_finalize(G64, n, mode == 2 ? d_gradE : nullptr, d_G, s))) return rc;
    return SMX_OK;
}

int smx_triplet_energy(const float *d_X, int64_t n, int64_t ldx, const smx_pot *pot, int map, double *d_E,
                       void *d_ws, size_t ws_bytes, int64_t *d_stats, void *stream) {
    return triplet_run(0, d_X, n, ldx, pot, map, d_E, nullptr, nullptr, d_ws, ws_bytes, d_stats, stream);
}

int smx_triplet_energy_grad(const float *d_X, int64_t n, int64_t ldx, const smx_pot *pot, int map,
                            double *d_E, float *d_G, void *d_ws, size_t ws_bytes, void *stream) {
    return triplet_run(1, d_X, n, ldx, pot, map, d_E, d_G, nullptr, d_ws, ws_bytes, nullptr, stream);
}

int smx_triplet_energy_backward(const float *d_X, int64_t n, int64_t ldx, const smx_pot *pot, int map,
                                const double *d_gradE, float *d_dX, void *d_ws, size_t ws_bytes,
                                void *stream) {
    return triplet_run(2, d_X, n, ldx, pot, map, nullptr, d_dX, d_gradE, d_ws, ws_bytes, nullptr, stream);
}

// ------------------------------------------------- allocation-free variant
// Workspace of smx_triplet_energy_grad_noalloc: a file-scope device array.  In
// host code its name is a host-side stand-in, not a device address; the
// address is taken per device with hipGetSymbolAddress (each GPU holds its own
// copy) and only that address is passed on.
constexpr int64_t kNoallocMaxN = SMX_NOALLOC_MAX_N;
constexpr size_t kNoallocBytes = 3 * kSlotBytes + size_t(kNoallocMaxN) * 3 * 8;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device, looked up on the first
// call per device; nullptr (with the error recorded) on failure.
static void *scratch_for_current_device() {
    int dev = -1;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        fail(SMX_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        fail(SMX_EUNSUPPORTED, "device %d is past the %d devices the static scratch supports", dev, kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        const hipError_t r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (r != hipSuccess || p == nullptr) {
            fail(SMX_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(r));
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

int smx_triplet_energy_grad_noalloc(const float *d_X, int64_t n, int64_t ldx, const smx_pot *pot, int map,
                                    double *d_E, float *d_G, void *stream) {
    if (n > kNoallocMaxN)
        return fail(SMX_EINVAL, "n = %lld exceeds the static scratch limit of %lld particles "
                    "(smx_triplet_energy_grad takes a workspace of any size)",
                    (long long)n, (long long)kNoallocMaxN);
    static_assert(kNoallocBytes >= 3 * kSlotBytes + size_t(kNoallocMaxN) * 3 * 8, "scratch holds trip_ws(max n)");
    return triplet_run(1, d_X, n, ldx, pot, map, d_E, d_G, nullptr, nullptr, 0, nullptr, stream, true);
}

int smx_probe_valu(float *d_out, int64_t blocks, int iters, void *stream) {
    if (d_out == nullptr) return fail(SMX_EINVAL, "out must not be NULL");
    if (blocks < 1 || blocks > (int64_t(1) << 24)) return fail(SMX_EINVAL, "blocks must be in [1, 2^24]");
    if (iters < 1) return fail(SMX_EINVAL, "iters must be >= 1");
    return launch_valu_probe(d_out, blocks, iters, S(stream));
}

int smx_simplex_life(const uint8_t *d_in, uint8_t *d_out, int64_t n, int map, int64_t *d_stats, void *d_ws,
                     size_t ws_bytes, void *stream) {
    if (n < 0) return fail(SMX_EINVAL, "n must be >= 0");
    if (n > (int64_t(1) << 24)) return fail(SMX_EOVERFLOW, "n = %lld exceeds 2^24", (long long)n);
    if (map < 0 || map > MAP_REC_LAUNCH) return fail(SMX_EINVAL, "unknown map %d", map);
    if (n > 0 && (d_in == nullptr || d_out == nullptr)) return fail(SMX_EINVAL, "in and out must not be NULL");
    if (n > 0 && d_in == d_out) return fail(SMX_EINVAL, "in and out must be different buffers");
    if (d_stats != nullptr && (d_ws == nullptr || ws_bytes < kSlotBytes))
        return fail(SMX_EINVAL, "statistics need a workspace of %zu bytes", kSlotBytes);
    MapGeom g{};
    if (n > 0 && !make_geom(2, (n + kLifeTile - 1) / kLifeTile, map, g)) return g_status;
    unsigned long long *slots = d_stats ? reinterpret_cast<unsigned long long *>(d_ws) : nullptr;
    int rc;
    if (slots && (rc = launch_fill_u64(reinterpret_cast<uint64_t *>(slots), kSlotBytes / 8, S(stream)))) return rc;
    if (n > 0 && (rc = launch_life(g, d_in, d_out, n, slots, S(stream)))) return rc;
    if (slots) return launch_stats_finalize(slots, g.G, d_stats, S(stream));
    return SMX_OK;
}

int smx_check_flags(uint32_t *flags, int clear) {
    if (flags == nullptr) return fail(SMX_EINVAL, "flags must not be NULL");
    if (!SMX_CHECKED) return fail(SMX_EUNSUPPORTED, "this library is built without device checks");
    const bool c = clear != 0;
    const unsigned parts[] = {check_flags_edm(c),  check_flags_gram(c),    check_flags_map(c),
                              check_flags_quad(c), check_flags_tripack(c), check_flags_triplet(c),
                              check_flags_life(c)};
    unsigned v = 0;
    for (unsigned p : parts) {
        if (p == ~0u) return fail(SMX_EHIP, "reading the device check flags failed");
        v |= p;
    }
    *flags = v;
    return SMX_OK;
}

int smx_quad_contacts(const float *d_X, int64_t n, int64_t ldx, double rc, int map, int64_t *d_count,
                      void *d_ws, size_t ws_bytes, int64_t *d_stats, void *stream) {
    if (n < 0) return fail(SMX_EINVAL, "n must be >= 0");
    if (n > 16384) return fail(SMX_EOVERFLOW, "n = %lld exceeds 16384", (long long)n);
    if (ldx < 3) return fail(SMX_EINVAL, "ldx (%lld) < 3", (long long)ldx);
    if (map < 0 || map > MAP_REC_LAUNCH) return fail(SMX_EINVAL, "unknown map %d", map);
    if (map == MAP_BELOW) return fail(SMX_EUNSUPPORTED, "the from-below map is defined for m = 2 and 3 only");
    if (!(rc >= 0.0) || !(rc < 1e18)) return fail(SMX_EINVAL, "rc must be finite and >= 0");
    if (d_count == nullptr) return fail(SMX_EINVAL, "count must not be NULL");
    if (n >= 4 && d_X == nullptr) return fail(SMX_EINVAL, "X must not be NULL");
    const QuadWs w = quad_ws(n);
    if (d_ws == nullptr || ws_bytes < w.total)
        return fail(SMX_EINVAL, "workspace of %zu bytes required (got %zu)", w.total, ws_bytes);
    MapGeom g2{}, g4{};
    if (n >= 4 && (!make_geom(2, w.nb, map, g2) || !make_geom(4, w.nb, map, g4))) return g_status;
    char *ws = reinterpret_cast<char *>(d_ws);
    unsigned long long *cslots = reinterpret_cast<unsigned long long *>(ws + w.cslots);
    unsigned long long *sslots = d_stats ? reinterpret_cast<unsigned long long *>(ws + w.sslots) : nullptr;
    uint64_t *W = reinterpret_cast<uint64_t *>(ws + w.words);
    int rc_;
    if ((rc_ = launch_fill_u64(reinterpret_cast<uint64_t *>(ws), 2 * kSlotBytes / 8, S(stream)))) return rc_;
    if (n >= 4) {
        const float rc2 = float(rc * rc);
        if ((rc_ = launch_contact_words(g2, d_X, n, ldx, rc2, W, w.npad, S(stream)))) return rc_;
        if ((rc_ = launch_quad(g4, W, w.npad, n, cslots, sslots, S(stream)))) return rc_;
    }
    if ((rc_ = launch_count_finalize(cslots, d_count, S(stream)))) return rc_;
    if (sslots) return launch_stats_finalize(sslots, g4.G, d_stats, S(stream));
    return SMX_OK;
}

static int triplet_packed_run(bool tiled, const float *d_X, int64_t n, int64_t ldx, double nu, int map, float *d_E,
                              void *d_ws, size_t ws_bytes, int64_t *d_stats, void *stream) {
    if (n < 0) return fail(SMX_EINVAL, "n must be >= 0");
    if (n > (int64_t(1) << 21)) return fail(SMX_EOVERFLOW, "n = %lld exceeds 2^21 (C(n,3) must fit 63 bits)", (long long)n);
    if (ldx < 3) return fail(SMX_EINVAL, "ldx (%lld) < 3", (long long)ldx);
    if (map < 0 || map > MAP_REC_LAUNCH) return fail(SMX_EINVAL, "unknown map %d", map);
    if (d_stats != nullptr && (d_ws == nullptr || ws_bytes < kSlotBytes))
        return fail(SMX_EINVAL, "statistics need a workspace of %zu bytes", kSlotBytes);
    if (n >= 3 && (d_X == nullptr || d_E == nullptr)) return fail(SMX_EINVAL, "X and E must not be NULL");
    MapGeom g{};
    if (n >= 3 && !make_geom(3, (n + kTripTile - 1) / kTripTile, map, g)) return g_status;
    unsigned long long *slots = d_stats ? reinterpret_cast<unsigned long long *>(d_ws) : nullptr;
    int rc;
    if (slots && (rc = launch_fill_u64(reinterpret_cast<uint64_t *>(slots), kSlotBytes / 8, S(stream)))) return rc;
    if (n >= 3 && (rc = launch_triplet_packed(g, d_X, n, ldx, float(nu), d_E, slots, tiled, S(stream)))) return rc;
    if (slots) return launch_stats_finalize(slots, g.G, d_stats, S(stream));
    return SMX_OK;
}

int smx_triplet_packed(const float *d_X, int64_t n, int64_t ldx, double nu, int map, float *d_E, void *d_ws,
                       size_t ws_bytes, int64_t *d_stats, void *stream) {
    return triplet_packed_run(false, d_X, n, ldx, nu, map, d_E, d_ws, ws_bytes, d_stats, stream);
}

int smx_triplet_packed_tiled(const float *d_X, int64_t n, int64_t ldx, double nu, int map, float *d_E, void *d_ws,
                             size_t ws_bytes, int64_t *d_stats, void *stream) {
    return triplet_packed_run(true, d_X, n, ldx, nu, map, d_E, d_ws, ws_bytes, d_stats, stream);
}

int smx_scale_grad(const float *d_G, int64_t n, const double *d_gradE, float *d_out, void *stream) {
    if (n < 0) return fail(SMX_EINVAL, "n must be >= 0");
    if (n > kMaxN) return fail(SMX_EOVERFLOW, "n exceeds 2^31 - 1");
    if (n == 0) return SMX_OK;
    if (d_G == nullptr || d_gradE == nullptr || d_out == nullptr) return fail(SMX_EINVAL, "NULL argument");
    return launch_scale_grad(d_G, n, d_gradE, d_out, S(stream));
}

int smx_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof = on != 0;
    return SMX_OK;
}

int smx_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    prof_collect();
    for (int k = 0; k < K_COUNT; ++k) {
        g_tot[k] = 0.0;
        g_cnt[k] = 0;
    }
    return SMX_OK;
}

int smx_profile_read(int kernel_id, double *total_ms, int64_t *launches) {
    if (kernel_id < 0 || kernel_id >= K_COUNT) return fail(SMX_EINVAL, "unknown kernel id %d", kernel_id);
    std::lock_guard<std::mutex> lk(g_mu);
    prof_collect();
    if (total_ms) *total_ms = g_tot[kernel_id];
    if (launches) *launches = g_cnt[kernel_id];
    return SMX_OK;
}

}  // extern "C"
