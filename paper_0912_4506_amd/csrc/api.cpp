// Host side of libjacobi.so: the C ABI of include/jacobi.h.
//
// Every entry point validates its arguments before it makes any HIP call, so
// the checks (and their error messages) are testable without a GPU.  Then it
// plans the passes and enqueues kernels on the caller's stream.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cctype>
#include <climits>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include <unistd.h>

#include "jacobi.h"
#include "kernels.h"
#include "lbm.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *where)
{
    return fail(JAC_EHIP, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
}

size_t elem_size(int dtype) { return dtype == JAC_F64 ? 8 : 4; }

// Checked, normalised geometry.
struct Geo {
    int64_t nx, ny, nz, sy, sz;
    int64_t span;  // elements from the first to one past the last element
};

int check_dtype(int dtype)
{
    if (dtype != JAC_F32 && dtype != JAC_F64)
        return fail(JAC_EARG, "dtype must be JAC_F32 (0) or JAC_F64 (1), got %d", dtype);
    return JAC_OK;
}

int check_grid(const jac_grid_t *g, Geo *out)
{
    if (!g)
        return fail(JAC_EARG, "grid descriptor is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(JAC_EARG, "interior extents must be >= 1, got %lld x %lld x %lld",
                    (long long)g->nx, (long long)g->ny, (long long)g->nz);
    // kernels index planes and rows with 32-bit ints
    if (g->nx > (1 << 28) || g->ny > (1 << 28) || g->nz > (1 << 28))
        return fail(JAC_EARG, "interior extents above 2^28 are not supported");
    Geo r;
    r.nx = g->nx;
    r.ny = g->ny;
    r.nz = g->nz;
    r.sy = g->sy ? g->sy : g->nx + 2;
    r.sz = g->sz ? g->sz : r.sy * (g->ny + 2);
    if (r.sy < r.nx + 2)
        return fail(JAC_EARG, "sy = %lld is below nx+2 = %lld", (long long)r.sy, (long long)(r.nx + 2));
    if (r.sz < r.sy * (r.ny + 2))
        return fail(JAC_EARG, "sz = %lld is below sy*(ny+2) = %lld", (long long)r.sz,
                    (long long)(r.sy * (r.ny + 2)));
    const long double span = (long double)(r.nz + 1) * r.sz + (long double)(r.ny + 1) * r.sy + r.nx + 2;
    if (span > (long double)(INT64_MAX / 16))
        return fail(JAC_EARG, "grid too large");
    r.span = (r.nz + 1) * r.sz + (r.ny + 1) * r.sy + r.nx + 2;
    *out = r;
    return JAC_OK;
}

int check_ptr(const void *p, int dtype, const char *name)
{
    if (!p)
        return fail(JAC_EARG, "%s is NULL", name);
    if ((uintptr_t)p % elem_size(dtype))
        return fail(JAC_EARG, "%s is not aligned to its element size", name);
    return JAC_OK;
}

bool overlap(const void *a, size_t abytes, const void *b, size_t bbytes)
{
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

jac::GridArgs grid_args(const Geo &g)
{
    return jac::GridArgs{g.nx, g.ny, g.nz, g.sy, g.sz};
}

// ------------------------------------------------------------- device facts --
struct DeviceFacts {
    int cus = 256;
    size_t lds_per_block = 160 * 1024;
    std::string arch = "gfx950";  // architecture name without feature flags
};

DeviceFacts device_facts()
{
    // queried once per process for the current device; falls back to MI355X
    // figures when no device is visible (argument checks still run)
    static std::once_flag once;
    static DeviceFacts f;
    std::call_once(once, [] {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            if (prop.multiProcessorCount > 0)
                f.cus = prop.multiProcessorCount;
            if (prop.sharedMemPerBlock > 0)
                f.lds_per_block = prop.sharedMemPerBlock;
            std::string name(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof prop.gcnArchName));
            name = name.substr(0, name.find(':'));
            if (!name.empty())
                f.arch = name;
        }
    });
    return f;
}

// JACOBI_DEBUG=1 in the environment prints every pass plan to stderr.
bool debug_plans()
{
    static const bool on = [] {
        const char *v = getenv("JACOBI_DEBUG");
        return v && *v && *v != '0';
    }();
    return on;
}

// --------------------------------------------------------------- tile menu --
const jac::TileShape kMenu[] = {
#define JAC_ROW(ID, CI, R, W) jac::TileShape{ID, CI, R, W},
    JAC_TILE_MENU(JAC_ROW)
#undef JAC_ROW
};
const int kMenuN = (int)(sizeof kMenu / sizeof kMenu[0]);

// The menu entry of block shape bx x by with `waves` waves per workgroup
// (0: the first such entry).
const jac::TileShape *find_shape(int bx, int by, int waves = 0)
{
    for (int n = 0; n < kMenuN; ++n)
        if (kMenu[n].bx() == bx && kMenu[n].by() == by && (waves == 0 || kMenu[n].waves == waves))
            return &kMenu[n];
    return nullptr;
}

int even_up(int v) { return (v + 1) & ~1; }

// Geometry of one temporally blocked pass at depth t with block shape s.
// (For a single-grid pass nkc is the number of workgroups and kchunk their
// share of planes; for a batch grid they are the k chunks of its blocks.)
struct TbPlan {
    const jac::TileShape *shape;
    int t;
    int hi, nti, ntj, nkc, kchunk;
    int64_t blocks() const { return nkc; }
};

// Blocks along one axis of n interior cells for blocks w wide with halo h:
// block 0 is valid on [1, w-h), every further block on w-2h more cells.
int64_t axis_blocks(int64_t n, int w, int h)
{
    const int64_t first = w - h, mid = w - 2 * h;
    if (first >= n + 1)
        return 1;
    return 1 + (n + 1 - first + mid - 1) / mid;
}

// Blocks along i and j for shape s at depth t; false if a block has no
// valid cells at this depth.
bool plan_ij(const Geo &g, const jac::TileShape &s, int t, TbPlan *p)
{
    p->shape = &s;
    p->t = t;
    p->hi = (s.ci % 2 == 0) ? even_up(t) : t;  // even first i keeps CI-wide pairs aligned
    if (s.bx() - 2 * p->hi < 1 || s.by() - 2 * t < 1)
        return false;
    const int64_t ni = axis_blocks(g.nx, s.bx(), p->hi), nj = axis_blocks(g.ny, s.by(), t);
    if (ni > INT_MAX / 2 || nj > INT_MAX / 2)
        return false;
    p->nti = (int)ni;
    p->ntj = (int)nj;
    return true;
}

// Split k so that the blocks fill the chip: minimise the modelled time
// ceil(blocks / slots) * (kchunk + 2t + c0), the number of rounds times the
// stream length of one block (a chunk streams 2t planes more than it writes)
// plus a fixed start-up cost c0 of about 12 stream steps per block (measured
// on 512^3 FP64 runs: one round of 256-plane chunks beats four rounds of
// 57-plane chunks that the model without c0 prefers by 2%).
void plan_k(const Geo &g, int slots, TbPlan *p, int kchunk_req)
{
    const int64_t nij = (int64_t)p->nti * p->ntj;
    if (kchunk_req > 0) {
        p->kchunk = (int)std::min<int64_t>(kchunk_req, g.nz);
    } else {
        double best = 1e300;
        int64_t best_kc = g.nz;
        const int64_t nmax = std::min<int64_t>(g.nz, 4096);
        for (int64_t n = 1; n <= nmax; ++n) {
            const int64_t kc = (g.nz + n - 1) / n;
            if ((g.nz + kc - 1) / kc != n)
                continue;  // same chunking as a smaller n
            const int64_t rounds = (nij * n + slots - 1) / slots;
            const double cost = (double)rounds * (double)(kc + 2 * p->t + 12);
            if (cost < best * (1 - 1e-9)) {
                best = cost;
                best_kc = kc;
            }
        }
        p->kchunk = (int)best_kc;
    }
    const int64_t nkc = (g.nz + p->kchunk - 1) / p->kchunk;
    p->nkc = (int)std::min<int64_t>(nij * nkc, INT_MAX);  // workgroups of the launch
}

// ---------------------------------------------------------- tuning cache --
// Choices made by jacobi_autotune (or read from a cache file), per (GPU
// architecture, dtype, geometry, T).  A file named by JACOBI_TUNE_CACHE is
// read at the first lookup and rewritten after every autotuning run.
using TuneKey = std::tuple<std::string, int, int64_t, int64_t, int64_t, int64_t, int64_t, int>;
struct TuneEntry {
    jac_tile_t tile;
    float ms;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

const char *tune_env_path()
{
    const char *p = getenv("JACOBI_TUNE_CACHE");
    return p && *p ? p : nullptr;
}

// One line of a cache file: "arch dtype nx ny nz sy sz T t bx by waves kchunk ms".
bool parse_tune_line(const char *line, TuneKey *key, TuneEntry *val, std::string *why)
{
    char arch[64], dt[8];
    long long nx, ny, nz, sy, sz;
    int T, t, bx, by, waves, kchunk, used = 0;
    float ms;
    if (sscanf(line, "%63s %7s %lld %lld %lld %lld %lld %d %d %d %d %d %d %f %n", arch, dt, &nx, &ny,
               &nz, &sy, &sz, &T, &t, &bx, &by, &waves, &kchunk, &ms, &used) != 14 ||
        line[used] != '\0') {
        *why = "expected: arch dtype nx ny nz sy sz T t bx by waves kchunk ms";
        return false;
    }
    for (const char *c = arch; *c; ++c)
        if (!isalnum((unsigned char)*c) && *c != '_' && *c != '-' && *c != '+') {
            *why = "bad architecture name";
            return false;
        }
    const int dtype = strcmp(dt, "f64") == 0 ? JAC_F64 : strcmp(dt, "f32") == 0 ? JAC_F32 : -1;
    if (dtype < 0) {
        *why = "dtype must be f32 or f64";
        return false;
    }
    const jac_grid_t g{nx, ny, nz, sy, sz};
    Geo geo;
    if (check_grid(&g, &geo) != JAC_OK || geo.sy != sy || geo.sz != sz) {
        *why = "bad geometry";
        return false;
    }
    if (T < 1 || t < 1 || t > JAC_MAX_DEPTH || t > T || kchunk < 0 || !(ms >= 0.f) ||
        !find_shape(bx, by, waves) || waves == 0) {
        *why = "T, t, block shape, kchunk or time out of range";
        return false;
    }
    *key = TuneKey{arch, dtype, nx, ny, nz, sy, sz, T};
    *val = TuneEntry{jac_tile_t{t, bx, by, kchunk, waves}, ms};
    return true;
}

// Reads a cache file; all lines or none are added.  Caller holds g_tune_mu.
int load_tune_file(const char *path, int *n_loaded)
{
    FILE *f = fopen(path, "r");
    if (!f)
        return fail(JAC_EARG, "cannot open %s", path);
    std::vector<std::pair<TuneKey, TuneEntry>> got;
    char line[512];
    int lineno = 0, rc = JAC_OK;
    while (fgets(line, sizeof line, f)) {
        ++lineno;
        size_t n = strlen(line);
        if (n + 1 == sizeof line && line[n - 1] != '\n') {
            rc = fail(JAC_EARG, "%s:%d: line too long", path, lineno);
            break;
        }
        while (n && (line[n - 1] == '\n' || line[n - 1] == '\r' || line[n - 1] == ' '))
            line[--n] = '\0';
        const char *p = line;
        while (*p == ' ' || *p == '\t')
            ++p;
        if (*p == '\0' || *p == '#')
            continue;
        TuneKey k;
        TuneEntry v;
        std::string why;
        if (!parse_tune_line(p, &k, &v, &why)) {
            rc = fail(JAC_EARG, "%s:%d: %s", path, lineno, why.c_str());
            break;
        }
        got.emplace_back(k, v);
    }
    if (rc == JAC_OK && ferror(f))
        rc = fail(JAC_EARG, "error reading %s", path);
    fclose(f);
    if (rc != JAC_OK)
        return rc;
    for (const auto &kv : got)
        g_tune[kv.first] = kv.second;
    if (n_loaded)
        *n_loaded = (int)got.size();
    return JAC_OK;
}

// Writes every remembered choice to path (via a temporary file and a rename).
// Caller holds g_tune_mu.
int save_tune_file(const char *path)
{
    const std::string tmp = std::string(path) + ".tmp." + std::to_string((long long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f)
        return fail(JAC_EARG, "cannot write %s", tmp.c_str());
    bool ok = fprintf(f, "# jacobi autotuning choices, format 1\n"
                         "# arch dtype nx ny nz sy sz T t bx by waves kchunk ms\n") > 0;
    for (const auto &kv : g_tune) {
        const TuneKey &k = kv.first;
        const jac_tile_t &c = kv.second.tile;
        ok = ok && fprintf(f, "%s %s %lld %lld %lld %lld %lld %d %d %d %d %d %d %.6g\n",
                           std::get<0>(k).c_str(), std::get<1>(k) == JAC_F64 ? "f64" : "f32",
                           (long long)std::get<2>(k), (long long)std::get<3>(k),
                           (long long)std::get<4>(k), (long long)std::get<5>(k),
                           (long long)std::get<6>(k), std::get<7>(k), c.t, c.bx, c.by, c.waves,
                           c.kchunk, (double)kv.second.ms) > 0;
    }
    ok = (fclose(f) == 0) && ok;
    if (!ok || rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return fail(JAC_EARG, "cannot write %s", path);
    }
    return JAC_OK;
}

// The JACOBI_TUNE_CACHE file, read once (a file that does not exist yet is
// no error; one that does not parse is reported on stderr and ignored).
void load_env_tune_once()
{
    static std::once_flag once;
    std::call_once(once, [] {
        const char *path = tune_env_path();
        if (!path)
            return;
        FILE *probe = fopen(path, "r");
        if (!probe)
            return;
        fclose(probe);
        const std::string saved = g_err;
        if (load_tune_file(path, nullptr) != JAC_OK)
            fprintf(stderr, "libjacobi: ignoring the tuning cache: %s\n", g_err.c_str());
        g_err = saved;
    });
}

bool tuned(int dtype, const Geo &g, int T, jac_tile_t *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_tune_once();
    auto it = g_tune.find(TuneKey{device_facts().arch, dtype, g.nx, g.ny, g.nz, g.sy, g.sz, T});
    if (it == g_tune.end())
        return false;
    *out = it->second.tile;
    return true;
}

// What a blocking choice is for: the kind of kernel it selects.
enum { KIND_PLAIN = 0, KIND_RHS = 1, KIND_TRACE = 2, KIND_BATCH = 3 };

// Untuned default depth, from 512^3 (single grid), 768^3 (right-hand side),
// 256^3 adjoint and 64-grid batch runs on MI355X.
int default_depth(int dtype, int kind)
{
    if (dtype == JAC_F64)
        return kind == KIND_BATCH ? 5 : 4;
    return kind == KIND_TRACE ? 3 : kind == KIND_PLAIN ? 6 : kind == KIND_RHS ? 7 : 5;
}

// Per-lane scratch bytes (register spills) of the kernel a choice selects;
// -1 when unknown (no device visible).
int kind_scratch(int dtype, int kind, int cfg, int depth)
{
    if (kind == KIND_BATCH)
        return jac::batched_scratch(dtype, cfg, depth, 0);
    const int mode = kind == KIND_RHS ? jac::MODE_RHS : kind == KIND_TRACE ? jac::MODE_TRACE
                                                                          : jac::MODE_PLAIN;
    return jac::tblock_scratch(dtype, cfg, depth, mode);
}

// Block shapes measured fastest on MI355X at a given depth: 512^3 sweeps
// without a right-hand side (T = 100; FP64 depth 5 also at 768^3, where it is
// the best depth), 768^3 FP32 sweeps with one (T = 50) and adjoint passes at
// 256^3 (T = 32: FP64 1.23 ms at depth 4 with 64x60 blocks of 12 waves, FP32
// 0.76 ms at depth 3 with the same blocks).
struct MeasuredShape {
    int dtype, kind, t, bx, by, waves;
};
const MeasuredShape kMeasured[] = {
    {JAC_F64, KIND_PLAIN, 3, 64, 64, 8},  {JAC_F64, KIND_PLAIN, 4, 64, 72, 12},
    {JAC_F64, KIND_PLAIN, 5, 64, 60, 12}, {JAC_F64, KIND_PLAIN, 6, 64, 48, 8},
    {JAC_F32, KIND_PLAIN, 4, 64, 72, 12}, {JAC_F32, KIND_PLAIN, 5, 64, 80, 16},
    {JAC_F32, KIND_PLAIN, 6, 64, 80, 16}, {JAC_F32, KIND_PLAIN, 7, 64, 80, 16},
    {JAC_F32, KIND_PLAIN, 8, 64, 80, 16}, {JAC_F32, KIND_RHS, 2, 64, 80, 16},
    {JAC_F32, KIND_RHS, 3, 64, 80, 16},   {JAC_F32, KIND_RHS, 4, 64, 56, 8},
    {JAC_F32, KIND_RHS, 5, 64, 60, 12},   {JAC_F32, KIND_RHS, 6, 64, 60, 12},
    {JAC_F32, KIND_RHS, 7, 64, 64, 16},   {JAC_F32, KIND_RHS, 8, 64, 64, 16},
    // adjoint passes (trace mode), timed at 256^3, T = 32
    {JAC_F64, KIND_TRACE, 4, 64, 60, 12}, {JAC_F32, KIND_TRACE, 2, 64, 60, 12},
    {JAC_F32, KIND_TRACE, 3, 64, 60, 12},
};

// Untuned default block shape: the measured one for (dtype, kind, t) if there
// is one, else the first of a preference order that has valid cells at depth
// t and compiles without register spills for this kind of kernel.
const jac::TileShape &default_shape(int dtype, int kind, int t)
{
    for (const auto &m : kMeasured)
        if (m.dtype == dtype && m.kind == kind && m.t == t)
            if (const jac::TileShape *s = find_shape(m.bx, m.by, m.waves))
                return *s;
    static const int pref64[][3] = {{64, 56, 8},  {64, 48, 8},  {64, 48, 16},  {64, 64, 8},
                                    {64, 64, 16}, {128, 32, 8}, {128, 32, 16}, {64, 32, 8},
                                    {128, 24, 8}, {128, 16, 8}};
    static const int pref32[][3] = {{64, 64, 16}, {64, 64, 8},  {64, 56, 8},   {64, 48, 16},
                                    {64, 48, 8},  {128, 32, 8}, {128, 32, 16}, {64, 32, 8},
                                    {128, 24, 8}, {128, 16, 8}};
    for (const auto &p : dtype == JAC_F64 ? pref64 : pref32) {
        const jac::TileShape *s = find_shape(p[0], p[1], p[2]);
        if (!s)
            continue;
        const int hi = (s->ci % 2 == 0) ? even_up(t) : t;
        const int need = kind == KIND_BATCH ? 3 : 2;  // batches need valid width >= halo
        if (s->bx() - need * hi < (kind == KIND_BATCH ? 0 : 1) || s->by() - need * t < (kind == KIND_BATCH ? 0 : 1))
            continue;
        if (kind_scratch(dtype, kind, s->id, t) > 0)
            continue;
        return *s;
    }
    return kMenu[0];
}

// Largest LDS a depth-t block of shape s needs.
size_t shape_lds(int dtype, const jac::TileShape &s, int t)
{
    const size_t one = (size_t)s.waves * 2 * t * s.ci * 64 * elem_size(dtype);
    return 2 * one <= 159 * 1024 ? 2 * one : one;  // double-buffered when it fits
}

int resolve_tile(int dtype, const jac_tile_t *tile, int T, jac_tile_t *out, const Geo *geo = nullptr,
                 int kind = KIND_PLAIN)
{
    jac_tile_t r = tile ? *tile : jac_tile_t{0, 0, 0, 0, 0};
    jac_tile_t c;
    if (geo && r.t == 0 && r.bx == 0 && r.by == 0 && tuned(dtype, *geo, T, &c)) {
        if (r.kchunk == 0)
            r.kchunk = c.kchunk;
        r.t = c.t;
        r.bx = c.bx;
        r.by = c.by;
        r.waves = c.waves;
    }
    if (r.t < 0 || r.t > JAC_MAX_DEPTH)
        return fail(JAC_EARG, "blocking depth t = %d outside 0..%d", r.t, JAC_MAX_DEPTH);
    if (r.kchunk < 0)
        return fail(JAC_EARG, "kchunk = %d is negative", r.kchunk);
    if ((r.bx == 0) != (r.by == 0))
        return fail(JAC_EARG, "bx and by must both be 0 (library choice) or both set");
    if (r.waves < 0)
        return fail(JAC_EARG, "waves = %d is negative", r.waves);
    if (r.bx && !find_shape(r.bx, r.by, r.waves))
        return fail(JAC_EUNSUPPORTED,
                    "no kernel for block shape %d x %d with %d waves (see jacobi_tile_menu)", r.bx,
                    r.by, r.waves);
    if (r.t == 0)
        r.t = default_depth(dtype, kind);
    if (T > 0 && r.t > T)
        r.t = T;
    if (r.bx == 0) {
        const jac::TileShape &s = default_shape(dtype, kind, r.t);
        r.bx = s.bx();
        r.by = s.by();
        r.waves = s.waves;
    } else if (r.waves == 0) {
        r.waves = find_shape(r.bx, r.by)->waves;
    }
    *out = r;
    return JAC_OK;
}

// Per-level size of the compact shell-face arrays: 2(ny nz + nx nz + nx ny).
int64_t face_count(const Geo &g) { return 2 * (g.ny * g.nz + g.nx * g.nz + g.nx * g.ny); }

// Extra work of the adjoint around the passes: each pass records the values
// of its levels next to the shell (trace) and folds them into the running
// face sums S, in level order.
template <typename real>
struct TraceSink {
    real *trace = nullptr;
    real *S = nullptr;
    int64_t F = 0;
};

// Every pass of a temporally blocked run of T sweeps can run with this
// blocking: the block has valid cells and fits the LDS at each pass depth
// (the depths take at most two values).  Checked before anything is
// enqueued, so a refused request leaves every buffer untouched.
int check_tblock_plan(int dtype, const Geo &g, int T, const jac_tile_t &tile)
{
    const jac::TileShape *shape = find_shape(tile.bx, tile.by, tile.waves);
    if (!shape)
        return fail(JAC_EUNSUPPORTED, "no kernel for block shape %d x %d with %d waves", tile.bx,
                    tile.by, tile.waves);
    if (g.sz * (int64_t)elem_size(dtype) >= jac::kDropOffset)
        return fail(JAC_EUNSUPPORTED, "planes of 2 GiB or more are not supported by the blocked kernels");
    if (T <= 0)
        return JAC_OK;
    const int P = (T + tile.t - 1) / tile.t;
    const int dlo = T / P, dhi = dlo + (T % P ? 1 : 0);
    for (int depth : {dhi, dlo}) {
        TbPlan plan;
        if (!plan_ij(g, *shape, depth, &plan))
            return fail(JAC_EUNSUPPORTED, "block %d x %d has no valid cells at depth %d", tile.bx,
                        tile.by, depth);
        if (shape_lds(dtype, *shape, depth) + 1024 > device_facts().lds_per_block)
            return fail(JAC_EUNSUPPORTED, "block %d x %d at depth %d needs more LDS than the device has",
                        tile.bx, tile.by, depth);
    }
    return JAC_OK;
}

// Enqueue the passes of a temporally blocked run (after copying a's shell
// into b); *npasses receives the pass count.
template <typename real>
int run_tblock(const Geo &g, real *a, real *b, int T, const jac_tile_t &tile, int mode,
               const real *rhs, const TraceSink<real> &sink, hipStream_t st, int *npasses)
{
    const jac::TileShape *shape = find_shape(tile.bx, tile.by, tile.waves);
    const int dtype = sizeof(real) == 8 ? JAC_F64 : JAC_F32;
    const int P = (T + tile.t - 1) / tile.t;
    const DeviceFacts dev = device_facts();
    int rc;
    if ((rc = check_tblock_plan(dtype, g, T, tile)))
        return rc;
    hipError_t e = jac::launch_copy_shell<real>(a, b, grid_args(g), st);
    if (e != hipSuccess)
        return hip_fail(e, "shell copy");
    for (int pass = 0; pass < P; ++pass) {
        const int depth = T / P + (pass < T % P ? 1 : 0);
        TbPlan plan;
        if (!plan_ij(g, *shape, depth, &plan))
            return fail(JAC_EUNSUPPORTED, "block %d x %d has no valid cells at depth %d", tile.bx,
                        tile.by, depth);
        if (shape_lds(dtype, *shape, depth) + 1024 > dev.lds_per_block)
            return fail(JAC_EUNSUPPORTED, "block %d x %d at depth %d needs more LDS than the device has",
                        tile.bx, tile.by, depth);
        int occ = jac::tblock_occupancy(dtype, shape->id, depth, mode);
        if (occ < 1)
            occ = 1;
        plan_k(g, dev.cus * occ, &plan, tile.kchunk);
        if (plan.blocks() > INT_MAX)
            return fail(JAC_EUNSUPPORTED, "too many blocks");
        jac::TbArgs<real> args;
        args.src = (pass % 2 == 0) ? a : b;
        args.dst = (pass % 2 == 0) ? b : a;
        args.rhs = rhs;
        args.trace = sink.trace;
        args.sy = g.sy;
        args.sz = g.sz;
        args.nx = (int)g.nx;
        args.ny = (int)g.ny;
        args.nz = (int)g.nz;
        args.nti = plan.nti;
        args.ntj = plan.ntj;
        args.hi = plan.hi;
        args.fstride = sink.F;
        args.kchunk = plan.kchunk;
        if (debug_plans())
            fprintf(stderr,
                    "[jacobi] pass %d/%d depth %d block %dx%d w%d: columns %dx%d, k chunk %d planes, "
                    "%d workgroups, occupancy %d/CU, %d CUs\n",
                    pass + 1, P, depth, shape->bx(), shape->by(), shape->waves, plan.nti, plan.ntj,
                    plan.kchunk, plan.nkc, occ, dev.cus);
        e = jac::launch_tblock<real>(shape->id, depth, mode, args, (int)plan.blocks(), st);
        if (e != hipSuccess)
            return hip_fail(e, "tblock launch");
        if (mode == jac::MODE_TRACE) {
            e = jac::launch_faces<real>(jac::FACES_ACCUM, nullptr, nullptr, sink.S, sink.trace,
                                        grid_args(g), sink.F, depth, st);
            if (e != hipSuccess)
                return hip_fail(e, "face accumulation");
        }
    }
    *npasses = P;
    return JAC_OK;
}

size_t adjoint_ws_bytes(int dtype, const Geo &g, int t)
{
    return (size_t)(2 + t) * (size_t)face_count(g) * elem_size(dtype);
}

template <typename real>
int run_adjoint(const Geo &g, real *la, real *lb, int T, const jac_tile_t &tile, void *ws,
                hipStream_t st, int *npasses)
{
    const int64_t F = face_count(g);
    real *G = (real *)ws, *S = G + F, *TR = S + F;
    const jac::GridArgs ga = grid_args(g);
    hipError_t e;
    // refuse before the set-up below changes lam_a's shell faces
    int rc0;
    if ((rc0 = check_tblock_plan(sizeof(real) == 8 ? JAC_F64 : JAC_F32, g, T, tile)))
        return rc0;
    if ((e = jac::launch_faces<real>(jac::FACES_SAVE, la, G, nullptr, nullptr, ga, F, 0, st)) ||
        (e = jac::launch_faces<real>(jac::FACES_ZERO, la, nullptr, nullptr, nullptr, ga, F, 0, st)) ||
        (e = jac::launch_faces<real>(jac::FACES_CLEAR_SUM, nullptr, nullptr, S, nullptr, ga, F, 0, st)))
        return hip_fail(e, "adjoint set-up");
    TraceSink<real> sink;
    sink.trace = TR;
    sink.S = S;
    sink.F = F;
    int rc = run_tblock<real>(g, la, lb, T, tile, jac::MODE_TRACE, nullptr, sink, st, npasses);
    if (rc)
        return rc;
    real *res = (*npasses % 2) ? lb : la;
    if ((e = jac::launch_faces<real>(jac::FACES_FINALIZE, res, G, S, nullptr, ga, F, 0, st)))
        return hip_fail(e, "adjoint shell gradient");
    return JAC_OK;
}

// ---------------------------------------------------------- batched plans --
// Default k chunk (planes per item) of a pipelined plan: short slabs, so that
// the passes in flight work on data the caches still hold.
constexpr int PIPELINE_KCHUNK = 16;

size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

struct BatchSizes {
    int nitems = 0, ntiles = 0, maxpasses = 0;
};

// Per-grid plan of a batched run; false with the error set on failure.
struct GridPlan {
    Geo geo;
    TbPlan tp;
    int passes, tiles;
};

int plan_batch_grid(int dtype, const jac_grid_t *g, int T, const jac_tile_t &tile, GridPlan *gp,
                    int idx)
{
    int rc;
    if ((rc = check_grid(g, &gp->geo)))
        return fail(rc, "grid %d: %s", idx, jacobi_last_error());
    if (T < 0)
        return fail(JAC_EARG, "grid %d: T = %d is negative", idx, T);
    const jac::TileShape *shape = find_shape(tile.bx, tile.by, tile.waves);
    const int t = tile.t;
    if (shape_lds(dtype, *shape, t) + 1024 > device_facts().lds_per_block)
        return fail(JAC_EUNSUPPORTED, "block %d x %d at depth %d needs more LDS than the device has",
                    tile.bx, tile.by, t);
    if (!plan_ij(gp->geo, *shape, t, &gp->tp))
        return fail(JAC_EUNSUPPORTED, "block %d x %d has no valid cells at depth %d", tile.bx, tile.by, t);
    // a block's neighbours of the previous pass are the adjacent blocks only
    // when every valid width is at least the halo
    if (shape->bx() - 2 * gp->tp.hi < gp->tp.hi || shape->by() - 2 * t < t)
        return fail(JAC_EUNSUPPORTED, "block %d x %d is too small for depth %d in a batch", tile.bx,
                    tile.by, t);
    // default: whole columns up to 256 planes (fewer, longer items; on the
    // 64-grid workload 30% faster than 64-plane chunks)
    int64_t kc = tile.kchunk > 0 ? tile.kchunk : std::min<int64_t>(gp->geo.nz, 256);
    kc = std::max<int64_t>(kc, t);
    kc = std::min<int64_t>(kc, gp->geo.nz);
    gp->tp.kchunk = (int)kc;
    gp->tp.nkc = (int)((gp->geo.nz + kc - 1) / kc);
    if (gp->tp.nkc > 1 && gp->tp.kchunk < t)
        return fail(JAC_EUNSUPPORTED, "k chunk shorter than the depth");
    const int64_t tiles = (int64_t)gp->tp.nti * gp->tp.ntj * gp->tp.nkc;
    if (tiles > (1 << 24))
        return fail(JAC_EUNSUPPORTED, "grid %d needs too many blocks", idx);
    gp->tiles = (int)tiles;
    gp->passes = (T + t - 1) / t;
    return JAC_OK;
}

int check_pair(int dtype, const Geo &g, const void *a, const void *b)
{
    int rc;
    if ((rc = check_ptr(a, dtype, "a")) || (rc = check_ptr(b, dtype, "b")))
        return rc;
    const size_t bytes = (size_t)g.span * elem_size(dtype);
    if (overlap(a, bytes, b, bytes))
        return fail(JAC_EARG, "grids a and b overlap");
    return JAC_OK;
}

// ------------------------------------------------------- compressed grid --
// A compressed run keeps the grid in one array of (nx+2+S) x (ny+2+S) x
// (nz+2) cells, S = t, in two frames: frame 0 holds cell (i, j, k) at
// (i+S, j+S, k), frame 1 at (i, j, k).  Even passes read frame 0 and write
// frame 1, odd passes the reverse.  Each pass also needs copies of the planes
// around its inner k chunk boundaries (taken before the pass) and rewrites
// the shell in the frame it wrote from a saved copy.
struct CompPlan {
    const jac::TileShape *shape = nullptr;
    int S = 0, P = 0, kchunk = 0, nkc = 0, maxitems = 0;
    int64_t span = 0;                        // elements of the array
    size_t nints = 0, snap_off = 0, store_off = 0, bytes = 0;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Geometry of the frames: strides of the padded array (0 = dense).
int check_comp_grid(const jac_grid_t *g, int S, Geo *out)
{
    if (!g)
        return fail(JAC_EARG, "grid descriptor is NULL");
    jac_grid_t d = *g;
    if (d.sy == 0)
        d.sy = d.nx + 2 + S;
    if (d.sz == 0)
        d.sz = d.sy * (d.ny + 2 + S);
    int rc;
    if ((rc = check_grid(&d, out)))
        return rc;
    if (out->sy < out->nx + 2 + S)
        return fail(JAC_EARG, "sy = %lld is below nx+2+t = %lld", (long long)out->sy,
                    (long long)(out->nx + 2 + S));
    if (out->sz < out->sy * (out->ny + 2 + S))
        return fail(JAC_EARG, "sz = %lld is below sy*(ny+2+t) = %lld", (long long)out->sz,
                    (long long)(out->sy * (out->ny + 2 + S)));
    return JAC_OK;
}

int plan_compressed(int dtype, const jac_grid_t *g, int T, const jac_tile_t *tile, Geo *geo,
                    CompPlan *cp)
{
    if (!tile || tile->t < 1 || tile->t > JAC_MAX_DEPTH)
        return fail(JAC_EARG, "a compressed run needs tile->t in 1..%d (the frame shift is t)",
                    JAC_MAX_DEPTH);
    const int S = tile->t;
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_comp_grid(g, S, geo)))
        return rc;
    if (T < 0)
        return fail(JAC_EARG, "T = %d is negative", T);
    jac_tile_t want = *tile, tl;
    if ((rc = resolve_tile(dtype, &want, 0, &tl, nullptr, KIND_PLAIN)))
        return rc;
    const jac::TileShape *shape = find_shape(tl.bx, tl.by, tl.waves);
    if (shape->ci != 1)
        return fail(JAC_EUNSUPPORTED, "a compressed run needs a 64-wide block, not %d x %d", tl.bx,
                    tl.by);
    if (tl.kchunk > 0 && tl.kchunk < S)
        return fail(JAC_EARG, "kchunk = %d is below t = %d", tl.kchunk, S);
    if (geo->sz * (int64_t)elem_size(dtype) >= jac::kDropOffset)
        return fail(JAC_EUNSUPPORTED, "planes of 2 GiB or more are not supported by the blocked kernels");
    CompPlan c;
    c.shape = shape;
    c.S = S;
    c.P = T > 0 ? (T + S - 1) / S : 0;
    c.span = (geo->nz + 1) * geo->sz + (geo->ny + 1 + S) * geo->sy + geo->nx + 2 + S;
    // blocks per pass (the depths of the passes differ by at most one).  A
    // block's output may overwrite inputs of its nearest neighbours only,
    // which holds when every valid width is at least depth + S.
    int64_t nij = 0;
    for (int pass = 0; pass < std::min(c.P, 2); ++pass) {
        const int depth = T / c.P + (pass < T % c.P ? 1 : 0);
        TbPlan tp;
        if (!plan_ij(*geo, *shape, depth, &tp))
            return fail(JAC_EUNSUPPORTED, "block %d x %d has no valid cells at depth %d", tl.bx,
                        tl.by, depth);
        if (shape->bx() - 2 * tp.hi < depth + S || shape->by() - 2 * depth < depth + S)
            return fail(JAC_EUNSUPPORTED, "block %d x %d is too small for a compressed run at t = %d",
                        tl.bx, tl.by, S);
        nij = std::max<int64_t>(nij, (int64_t)tp.nti * tp.ntj);
    }
    // one k chunking for every pass, planned for depth t
    TbPlan tp;
    if (!plan_ij(*geo, *shape, S, &tp))
        return fail(JAC_EUNSUPPORTED, "block %d x %d has no valid cells at depth %d", tl.bx, tl.by,
                    S);
    int occ = jac::tblock_occupancy(dtype, shape->id, S, jac::MODE_COMP);
    plan_k(*geo, device_facts().cus * std::max(occ, 1), &tp, tl.kchunk);
    c.kchunk = std::max(tp.kchunk, S);
    c.nkc = (int)((geo->nz + c.kchunk - 1) / c.kchunk);
    if (nij * c.nkc > INT_MAX / 2)
        return fail(JAC_EUNSUPPORTED, "too many blocks");
    c.maxitems = (int)(nij * c.nkc);
    const size_t esz = elem_size(dtype);
    c.nints = 1 + (size_t)c.P * (1 + (size_t)c.maxitems);
    c.snap_off = align256(c.nints * sizeof(int));
    c.store_off = align256(c.snap_off + (size_t)(c.nkc - 1) * (2 * S + 1) * geo->sz * esz);
    c.bytes = c.store_off + (size_t)jac::shell_count(grid_args(*geo)) * esz;
    *cp = c;
    return JAC_OK;
}

template <typename real>
int run_compressed(const Geo &g, real *u, int T, const CompPlan &c, unsigned char *ws,
                   hipStream_t st)
{
    const int S = c.S;
    int *ints = (int *)ws;
    real *snap = (real *)(ws + c.snap_off);
    real *store = (real *)(ws + c.store_off);
    const int64_t off0 = S + S * g.sy;  // frame 0; frame 1 starts at u
    const jac::GridArgs ga = grid_args(g);
    hipError_t e;
    if ((e = jac::launch_zero_ints(ints, (int64_t)c.nints, st)) ||
        (e = jac::launch_shell_store<real>(1, u + off0, store, ga, st)))
        return hip_fail(e, "compressed set-up");
    for (int pass = 0; pass < c.P; ++pass) {
        const int depth = T / c.P + (pass < T % c.P ? 1 : 0);
        TbPlan tp;
        plan_ij(g, *c.shape, depth, &tp);
        const int64_t soff = pass % 2 == 0 ? off0 : 0, doff = pass % 2 == 0 ? 0 : off0;
        // planes [Kb - S, Kb + S] around each inner chunk boundary Kb
        for (int b = 1; b < c.nkc; ++b) {
            const int64_t kb = 1 + (int64_t)b * c.kchunk, lo = kb - S;
            const int64_t hi = std::min<int64_t>(kb + S, g.nz + 1);
            const int64_t n = std::min<int64_t>((hi - lo + 1) * g.sz, c.span - lo * g.sz);
            e = hipMemcpyAsync(snap + (int64_t)(b - 1) * (2 * S + 1) * g.sz, u + lo * g.sz,
                               (size_t)n * sizeof(real), hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess)
                return hip_fail(e, "boundary plane copy");
        }
        jac::TbArgs<real> args{};
        args.src = u + soff;
        args.dst = u + doff;
        args.sy = g.sy;
        args.sz = g.sz;
        args.nx = (int)g.nx;
        args.ny = (int)g.ny;
        args.nz = (int)g.nz;
        args.nti = tp.nti;
        args.ntj = tp.ntj;
        args.hi = tp.hi;
        args.kchunk = c.kchunk;
        args.snap = snap + soff;
        args.ticket = ints + 1 + (int64_t)pass * (1 + c.maxitems);
        args.prog = args.ticket + 1;
        args.error = ints;
        args.shift = S;
        args.dir = pass % 2 == 0 ? 1 : -1;
        args.spin_limit = 1 << 20;
        const int nblocks = tp.nti * tp.ntj * c.nkc;
        if (debug_plans())
            fprintf(stderr,
                    "[jacobi] compressed pass %d/%d depth %d block %dx%d w%d: columns %dx%d, "
                    "k chunk %d planes, %d workgroups\n",
                    pass + 1, c.P, depth, c.shape->bx(), c.shape->by(), c.shape->waves, tp.nti,
                    tp.ntj, c.kchunk, nblocks);
        if ((e = jac::launch_tblock<real>(c.shape->id, depth, jac::MODE_COMP, args, nblocks, st)))
            return hip_fail(e, "compressed pass launch");
        if ((e = jac::launch_shell_store<real>(0, u + doff, store, ga, st)))
            return hip_fail(e, "compressed shell");
    }
    return JAC_OK;
}

}  // namespace

// ====================================================================== ABI ==
extern "C" {

int jacobi_version(void) { return JACOBI_ABI_VERSION; }

const char *jacobi_last_error(void) { return g_err.c_str(); }

int jacobi_plain(int dtype, const jac_grid_t *g, void *a, void *b, int T, void *stream,
                 int *out_idx)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_grid(g, &geo)) ||
        (rc = check_pair(dtype, geo, a, b)))
        return rc;
    if (T < 0)
        return fail(JAC_EARG, "T = %d is negative", T);
    if (!out_idx)
        return fail(JAC_EARG, "out_idx is NULL");
    *out_idx = 0;
    if (T == 0)
        return JAC_OK;
    if (geo.sz * (int64_t)elem_size(dtype) >= jac::kDropOffset)
        return fail(JAC_EUNSUPPORTED, "planes of 2 GiB or more are not supported by the sweep kernels");
    hipStream_t st = (hipStream_t)stream;
    // k-chunk: long streams (contiguous reads), but enough blocks to fill the
    // chip (with 128-thread strips, two per CU); from there up to four times
    // as many chunks, the count with the least ceil(blocks / CUs) x (chunk
    // + 2 planes): blocks that spread evenly over the CUs (768^3: 2304
    // blocks, 9 per CU, instead of 576, 2.25 per CU, where a quarter of the
    // CUs run a third block: 199 -> 248 GLUP/s with 1728)
    const int nt = jac::plain_threads(geo.nx);
    const int64_t strips = ((geo.nx + 2 * nt - 1) / (2 * nt)) * ((geo.ny + 7) / 8);
    const int64_t cus = device_facts().cus;
    const int64_t slots = cus * (nt == 128 ? 2 : 1);
    int64_t nkc = (slots + strips - 1) / strips;
    nkc = std::max<int64_t>(1, std::min<int64_t>(nkc, geo.nz));
    {
        int64_t best = nkc;
        double best_cost = 1e300;
        for (int64_t n = nkc; n <= std::min<int64_t>(4 * nkc, geo.nz); ++n) {
            const int64_t kc = (geo.nz + n - 1) / n;
            if ((geo.nz + kc - 1) / kc != n)
                continue;  // the same chunking as a smaller count
            const double cost = (double)((strips * n + cus - 1) / cus) * (double)(kc + 2);
            if (cost < best_cost * (1 - 1e-9)) {
                best_cost = cost;
                best = n;
            }
        }
        nkc = best;
    }
    const int kchunk = (int)((geo.nz + nkc - 1) / nkc);
    jac::PlainArgs p{(int)geo.nx, (int)geo.ny, (int)geo.nz, kchunk, geo.sy, geo.sz};
    hipError_t e;
    if (dtype == JAC_F64)
        e = jac::launch_copy_shell<double>((const double *)a, (double *)b, grid_args(geo), st);
    else
        e = jac::launch_copy_shell<float>((const float *)a, (float *)b, grid_args(geo), st);
    if (e != hipSuccess)
        return hip_fail(e, "shell copy");
    for (int s = 0; s < T; ++s) {
        void *src = (s % 2 == 0) ? a : b;
        void *dst = (s % 2 == 0) ? b : a;
        if (dtype == JAC_F64)
            e = jac::launch_plain<double>((const double *)src, (double *)dst, p, st);
        else
            e = jac::launch_plain<float>((const float *)src, (float *)dst, p, st);
        if (e != hipSuccess)
            return hip_fail(e, "plain sweep launch");
    }
    *out_idx = T % 2;
    return JAC_OK;
}

int jacobi_tblock(int dtype, const jac_grid_t *g, void *a, void *b, int T, const jac_tile_t *tile,
                  const void *rhs, void *stream, int *out_idx)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_grid(g, &geo)) ||
        (rc = check_pair(dtype, geo, a, b)))
        return rc;
    if (T < 0)
        return fail(JAC_EARG, "T = %d is negative", T);
    if (!out_idx)
        return fail(JAC_EARG, "out_idx is NULL");
    if (rhs) {
        if ((rc = check_ptr(rhs, dtype, "rhs")))
            return rc;
        const size_t bytes = (size_t)geo.span * elem_size(dtype);
        if (overlap(rhs, bytes, a, bytes) || overlap(rhs, bytes, b, bytes))
            return fail(JAC_EARG, "rhs overlaps a or b");
    }
    jac_tile_t tl;
    if ((rc = resolve_tile(dtype, tile, T, &tl, rhs ? nullptr : &geo, rhs ? KIND_RHS : KIND_PLAIN)))
        return rc;
    *out_idx = 0;
    if (T == 0)
        return JAC_OK;
    const int mode = rhs ? jac::MODE_RHS : jac::MODE_PLAIN;
    int P = 0;
    if (dtype == JAC_F64)
        rc = run_tblock<double>(geo, (double *)a, (double *)b, T, tl, mode, (const double *)rhs,
                                TraceSink<double>(), (hipStream_t)stream, &P);
    else
        rc = run_tblock<float>(geo, (float *)a, (float *)b, T, tl, mode, (const float *)rhs,
                               TraceSink<float>(), (hipStream_t)stream, &P);
    if (rc)
        return rc;
    *out_idx = P % 2;
    return JAC_OK;
}

size_t jacobi_adjoint_workspace(int dtype, const jac_grid_t *g, int t)
{
    g_err.clear();
    Geo geo;
    if (check_dtype(dtype) || check_grid(g, &geo))
        return 0;
    if (t < 0 || t > JAC_MAX_DEPTH) {
        fail(JAC_EARG, "blocking depth t = %d outside 0..%d", t, JAC_MAX_DEPTH);
        return 0;
    }
    if (t == 0)
        t = JAC_MAX_DEPTH;  // room for any depth the library may choose
    return adjoint_ws_bytes(dtype, geo, t);
}

int jacobi_adjoint(int dtype, const jac_grid_t *g, void *lam_a, void *lam_b, int T,
                   const jac_tile_t *tile, void *ws, size_t ws_bytes, void *stream, int *out_idx)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_grid(g, &geo)) ||
        (rc = check_pair(dtype, geo, lam_a, lam_b)))
        return rc;
    if (T < 0)
        return fail(JAC_EARG, "T = %d is negative", T);
    if (!out_idx)
        return fail(JAC_EARG, "out_idx is NULL");
    jac_tile_t tl;
    if ((rc = resolve_tile(dtype, tile, T, &tl, nullptr, KIND_TRACE)))
        return rc;
    *out_idx = 0;
    if (T == 0)
        return JAC_OK;  // the gradient w.r.t. level 0 is the input itself
    // the trace pass addresses one level of face values with 32-bit byte offsets
    if (face_count(geo) * (int64_t)elem_size(dtype) > INT_MAX)
        return fail(JAC_EUNSUPPORTED, "one level of shell faces (%lld values) takes 2 GiB or more",
                    (long long)face_count(geo));
    const size_t need = adjoint_ws_bytes(dtype, geo, tl.t);
    if (!ws)
        return fail(JAC_EWORKSPACE, "workspace is NULL (%zu bytes needed)", need);
    if (ws_bytes < need)
        return fail(JAC_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
    if ((uintptr_t)ws % elem_size(dtype))
        return fail(JAC_EARG, "workspace is not aligned to the element size");
    const size_t gbytes = (size_t)geo.span * elem_size(dtype);
    if (overlap(ws, need, lam_a, gbytes) || overlap(ws, need, lam_b, gbytes))
        return fail(JAC_EARG, "workspace overlaps lam_a or lam_b");
    int P = 0;
    if (dtype == JAC_F64)
        rc = run_adjoint<double>(geo, (double *)lam_a, (double *)lam_b, T, tl, ws,
                                 (hipStream_t)stream, &P);
    else
        rc = run_adjoint<float>(geo, (float *)lam_a, (float *)lam_b, T, tl, ws,
                                (hipStream_t)stream, &P);
    if (rc)
        return rc;
    *out_idx = P % 2;
    return JAC_OK;
}

size_t jacobi_compressed_workspace(int dtype, const jac_grid_t *g, int T, const jac_tile_t *tile)
{
    g_err.clear();
    Geo geo;
    CompPlan c;
    if (plan_compressed(dtype, g, T, tile, &geo, &c))
        return 0;
    return c.bytes;
}

int jacobi_compressed(int dtype, const jac_grid_t *g, void *u, int T, const jac_tile_t *tile,
                      void *ws, size_t ws_bytes, void *stream, int *out_frame)
{
    g_err.clear();
    Geo geo;
    CompPlan c;
    int rc;
    if ((rc = plan_compressed(dtype, g, T, tile, &geo, &c)) || (rc = check_ptr(u, dtype, "u")))
        return rc;
    if (!out_frame)
        return fail(JAC_EARG, "out_frame is NULL");
    if (!ws)
        return fail(JAC_EWORKSPACE, "workspace is NULL (%zu bytes needed)", c.bytes);
    if (ws_bytes < c.bytes)
        return fail(JAC_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, c.bytes);
    if ((uintptr_t)ws % 256)
        return fail(JAC_EARG, "workspace is not 256-byte aligned");
    if (overlap(ws, c.bytes, u, (size_t)c.span * elem_size(dtype)))
        return fail(JAC_EARG, "workspace overlaps the grid");
    *out_frame = 0;
    if (T == 0)
        return JAC_OK;
    if (dtype == JAC_F64)
        rc = run_compressed<double>(geo, (double *)u, T, c, (unsigned char *)ws, (hipStream_t)stream);
    else
        rc = run_compressed<float>(geo, (float *)u, T, c, (unsigned char *)ws, (hipStream_t)stream);
    if (rc)
        return rc;
    *out_frame = c.P % 2;
    return JAC_OK;
}

size_t jacobi_residual_workspace(const jac_grid_t *g)
{
    g_err.clear();
    Geo geo;
    if (check_grid(g, &geo))
        return 0;
    return (size_t)jac::residual_partials(grid_args(geo)) * sizeof(double);
}

int jacobi_residual_f64(const jac_grid_t *g, const double *x, float *r32, double *norm2, void *ws,
                        size_t ws_bytes, void *stream)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_grid(g, &geo)) || (rc = check_ptr(x, JAC_F64, "x")) ||
        (rc = check_ptr(r32, JAC_F32, "r32")) || (rc = check_ptr(norm2, JAC_F64, "norm2")))
        return rc;
    const size_t need = (size_t)jac::residual_partials(grid_args(geo)) * sizeof(double);
    if (!ws)
        return fail(JAC_EWORKSPACE, "workspace is NULL (%zu bytes needed)", need);
    if (ws_bytes < need)
        return fail(JAC_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
    if ((uintptr_t)ws % 8)
        return fail(JAC_EARG, "workspace is not 8-byte aligned");
    const size_t xb = (size_t)geo.span * 8, rb = (size_t)geo.span * 4;
    if (overlap(x, xb, r32, rb) || overlap(ws, need, x, xb) || overlap(ws, need, r32, rb) ||
        overlap(norm2, 8, x, xb) || overlap(norm2, 8, r32, rb) || overlap(norm2, 8, ws, need))
        return fail(JAC_EARG, "x, r32, norm2 and the workspace must not overlap");
    hipError_t e = jac::launch_residual(x, r32, (double *)ws, norm2, grid_args(geo),
                                        (hipStream_t)stream);
    return e == hipSuccess ? JAC_OK : hip_fail(e, "residual launch");
}

int jacobi_residual_f64_noalloc(const jac_grid_t *g, const double *x, float *r32, double *norm2,
                                void *stream)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_grid(g, &geo)) || (rc = check_ptr(x, JAC_F64, "x")) ||
        (rc = check_ptr(r32, JAC_F32, "r32")) || (rc = check_ptr(norm2, JAC_F64, "norm2")))
        return rc;
    const size_t xb = (size_t)geo.span * 8, rb = (size_t)geo.span * 4;
    if (overlap(x, xb, r32, rb) || overlap(norm2, 8, x, xb) || overlap(norm2, 8, r32, rb))
        return fail(JAC_EARG, "x, r32 and norm2 must not overlap");
    const int64_t need = jac::residual_partials_plain(grid_args(geo));
    if (need > jac::noalloc_partials_max())
        return fail(JAC_EUNSUPPORTED,
                    "the grid needs %lld partial sums; the allocation-free residual holds at most "
                    "%lld (ceil(nx/256) * ceil(ny/8) * ceil(nz/64)); use jacobi_residual_f64 with "
                    "a workspace",
                    (long long)need, (long long)jac::noalloc_partials_max());
    double *partial = nullptr;
    hipError_t e = jac::noalloc_scratch(&partial);
    if (e != hipSuccess)
        return hip_fail(e, "scratch address");
    e = jac::launch_residual(x, r32, partial, norm2, grid_args(geo), (hipStream_t)stream);
    return e == hipSuccess ? JAC_OK : hip_fail(e, "residual launch");
}

int jacobi_update_residual_f64(const jac_grid_t *g, const double *x, const float *e32,
                               double *x_new, float *r32, float *zero32, double *norm2, void *ws,
                               size_t ws_bytes, void *stream)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_grid(g, &geo)) || (rc = check_ptr(x, JAC_F64, "x")) ||
        (rc = check_ptr(e32, JAC_F32, "e32")) || (rc = check_ptr(x_new, JAC_F64, "x_new")) ||
        (rc = check_ptr(r32, JAC_F32, "r32")) || (rc = check_ptr(zero32, JAC_F32, "zero32")) ||
        (rc = check_ptr(norm2, JAC_F64, "norm2")))
        return rc;
    const size_t need = (size_t)jac::residual_partials(grid_args(geo)) * sizeof(double);
    if (!ws)
        return fail(JAC_EWORKSPACE, "workspace is NULL (%zu bytes needed)", need);
    if (ws_bytes < need)
        return fail(JAC_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
    if ((uintptr_t)ws % 8)
        return fail(JAC_EARG, "workspace is not 8-byte aligned");
    const size_t xb = (size_t)geo.span * 8, fb = (size_t)geo.span * 4;
    const void *buf[] = {x, e32, x_new, r32, zero32, norm2, ws};
    const size_t len[] = {xb, fb, xb, fb, fb, 8, need};
    for (int u = 0; u < 7; ++u)
        for (int v = u + 1; v < 7; ++v)
            if (overlap(buf[u], len[u], buf[v], len[v]))
                return fail(JAC_EARG,
                            "x, e32, x_new, r32, zero32, norm2 and the workspace must not overlap");
    hipError_t e = jac::launch_update_residual(x, e32, x_new, zero32, r32, (double *)ws, norm2,
                                               grid_args(geo), (hipStream_t)stream);
    return e == hipSuccess ? JAC_OK : hip_fail(e, "update-residual launch");
}

int jacobi_update_f64(const jac_grid_t *g, double *x, const float *e32, void *stream)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_grid(g, &geo)) || (rc = check_ptr(x, JAC_F64, "x")) ||
        (rc = check_ptr(e32, JAC_F32, "e32")))
        return rc;
    if (overlap(x, (size_t)geo.span * 8, e32, (size_t)geo.span * 4))
        return fail(JAC_EARG, "x and e32 overlap");
    hipError_t e = jac::launch_update(x, e32, grid_args(geo), (hipStream_t)stream);
    return e == hipSuccess ? JAC_OK : hip_fail(e, "update launch");
}

int jacobi_fill(int dtype, const jac_grid_t *g, void *x, double value, void *stream)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_grid(g, &geo)) || (rc = check_ptr(x, dtype, "x")))
        return rc;
    hipError_t e = dtype == JAC_F64
                       ? jac::launch_grid_fill<double>((double *)x, value, grid_args(geo),
                                                       (hipStream_t)stream)
                       : jac::launch_grid_fill<float>((float *)x, (float)value, grid_args(geo),
                                                      (hipStream_t)stream);
    return e == hipSuccess ? JAC_OK : hip_fail(e, "fill launch");
}

int jacobi_grid_add(int dtype, const jac_grid_t *g, void *dst, const void *src, void *stream)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_grid(g, &geo)) ||
        (rc = check_ptr(dst, dtype, "dst")) || (rc = check_ptr(src, dtype, "src")))
        return rc;
    const size_t bytes = (size_t)geo.span * elem_size(dtype);
    if (dst != src && overlap(dst, bytes, src, bytes))
        return fail(JAC_EARG, "dst and src overlap (only dst == src may share memory)");
    const hipStream_t st = (hipStream_t)stream;
    hipError_t e = dtype == JAC_F64
                       ? jac::launch_grid_add<double>((double *)dst, (const double *)src, grid_args(geo), st)
                       : jac::launch_grid_add<float>((float *)dst, (const float *)src, grid_args(geo), st);
    return e == hipSuccess ? JAC_OK : hip_fail(e, "grid add launch");
}

static int batch_common(int dtype, int n, const jac_grid_t *g, const int *T, const jac_tile_t *tile,
                        jac_tile_t *tl, GridPlan **plans_out, BatchSizes *bs)
{
    int rc;
    if ((rc = check_dtype(dtype)))
        return rc;
    if (n < 1 || n > 65535)
        return fail(JAC_EARG, "batch size n = %d outside 1..65535", n);
    if (!g || !T)
        return fail(JAC_EARG, "grid or T array is NULL");
    int Tmax = 0;
    for (int m = 0; m < n; ++m)
        Tmax = std::max(Tmax, T[m]);
    if ((rc = resolve_tile(dtype, tile, Tmax, tl, nullptr, KIND_BATCH)))
        return rc;
    if (tl->t < 1)
        tl->t = 1;
    GridPlan *plans = new GridPlan[n];
    BatchSizes z;
    for (int m = 0; m < n; ++m) {
        if ((rc = plan_batch_grid(dtype, &g[m], T[m], *tl, &plans[m], m))) {
            delete[] plans;
            return rc;
        }
        if ((int64_t)z.nitems + (int64_t)plans[m].passes * plans[m].tiles > INT_MAX / 2 ||
            (int64_t)z.ntiles + plans[m].tiles > INT_MAX / 2) {
            delete[] plans;
            return fail(JAC_EUNSUPPORTED, "batch too large");
        }
        z.nitems += plans[m].passes * plans[m].tiles;
        z.ntiles += plans[m].tiles;
        z.maxpasses = std::max(z.maxpasses, plans[m].passes);
    }
    *plans_out = plans;
    *bs = z;
    return JAC_OK;
}

static size_t batch_image_bytes(int n, const BatchSizes &z)
{
    return align16(sizeof(jac::BatchHeader)) + align16((size_t)n * sizeof(jac::BatchGrid)) +
           align16((size_t)z.nitems * sizeof(jac::BatchItem)) +
           align16((size_t)(z.maxpasses + 1) * sizeof(int));
}

size_t jacobi_batched_plan_bytes(int dtype, int n, const jac_grid_t *g, const int *T,
                                 const jac_tile_t *tile)
{
    g_err.clear();
    jac_tile_t tl;
    GridPlan *plans = nullptr;
    BatchSizes z;
    if (batch_common(dtype, n, g, T, tile, &tl, &plans, &z))
        return 0;
    delete[] plans;
    return batch_image_bytes(n, z);
}

// Plan image of a batched run.  team = 0: items pass by pass.  team >= 1
// (one grid): the pipelined schedule of temporal blocking (Sect. 1.3)
// in GPU form.  The passes form segments of `team` consecutive passes; within
// a segment, wavefront w holds pass seg + s on k chunk w - s * (dl + 1), so
// pass p works dl + 1 chunks behind pass p-1 (one chunk of halo plus the
// lower distance), like the threads of a team following each other through
// the blocks of a shared cache.  Every counter an item waits on belongs to an
// earlier item in this order, which keeps the relaxed waits deadlock-free:
//  * the 27 neighbours of the previous pass (chunks tk-1..tk+1) and the
//    previous pass's chunk tk + dl: the same or an earlier wavefront,
//    earlier pass;
//  * the team delay: a segment's front pass waits on the previous
//    segment, all of which comes earlier;
//  * the upper bound, the next pass's chunk tk - du - 2: wavefront
//    w + dl - du - 1, earlier because du >= dl (checked); a segment's rear
//    pass does not wait on the next segment (which comes later).
static int build_plan(int dtype, int n, const jac_grid_t *g, void *const *a, void *const *b,
                      const int *T, const jac_tile_t *tile, void *plan_host, size_t plan_bytes,
                      int *out_idx_host, int team, const jac_pipeline_t &sync)
{
    jac_tile_t tl;
    GridPlan *plans = nullptr;
    BatchSizes z;
    int rc;
    if ((rc = batch_common(dtype, n, g, T, tile, &tl, &plans, &z)))
        return rc;
    auto done = [&](int code) {
        delete[] plans;
        return code;
    };
    if (!a || !b || !plan_host || !out_idx_host)
        return done(fail(JAC_EARG, "a, b, plan_host and out_idx_host must not be NULL"));
    const size_t need = batch_image_bytes(n, z);
    if (plan_bytes < need)
        return done(fail(JAC_EWORKSPACE, "plan buffer has %zu bytes, %zu needed", plan_bytes, need));
    const size_t es = elem_size(dtype);
    for (int m = 0; m < n; ++m) {
        if ((rc = check_pair(dtype, plans[m].geo, a[m], b[m])))
            return done(fail(rc, "grid %d: %s", m, jacobi_last_error()));
    }
    for (int m = 0; m < n; ++m)
        for (int q = m + 1; q < n; ++q) {
            const size_t bm = (size_t)plans[m].geo.span * es, bq = (size_t)plans[q].geo.span * es;
            if (overlap(a[m], bm, a[q], bq) || overlap(a[m], bm, b[q], bq) ||
                overlap(b[m], bm, a[q], bq) || overlap(b[m], bm, b[q], bq))
                return done(fail(JAC_EARG, "grids %d and %d overlap", m, q));
        }
    unsigned char *img = (unsigned char *)plan_host;
    memset(img, 0, need);
    jac::BatchHeader h;
    memset(&h, 0, sizeof h);
    h.magic = jac::BATCH_MAGIC;
    h.dtype = dtype;
    h.n = n;
    h.nitems = z.nitems;
    h.ntiles = z.ntiles;
    h.cfg = find_shape(tl.bx, tl.by, tl.waves)->id;
    h.t = tl.t;
    h.maxpasses = z.maxpasses;
    h.order = team > 0 ? 1 : 0;
    h.team = team;
    h.grids_off = (int64_t)align16(sizeof(jac::BatchHeader));
    h.items_off = h.grids_off + (int64_t)align16((size_t)n * sizeof(jac::BatchGrid));
    h.pass_off = h.items_off + (int64_t)align16((size_t)z.nitems * sizeof(jac::BatchItem));
    h.total_bytes = (int64_t)need;
    jac::BatchGrid *grids = (jac::BatchGrid *)(img + h.grids_off);
    jac::BatchItem *items = (jac::BatchItem *)(img + h.items_off);
    int *pass_start = (int *)(img + h.pass_off);
    int off = 0;
    for (int m = 0; m < n; ++m) {
        const GridPlan &gp = plans[m];
        jac::BatchGrid &G = grids[m];
        G.a = a[m];
        G.b = b[m];
        G.sy = gp.geo.sy;
        G.sz = gp.geo.sz;
        G.nx = (int)gp.geo.nx;
        G.ny = (int)gp.geo.ny;
        G.nz = (int)gp.geo.nz;
        G.nti = gp.tp.nti;
        G.ntj = gp.tp.ntj;
        G.nkc = gp.tp.nkc;
        G.hi = gp.tp.hi;
        G.kchunk = gp.tp.kchunk;
        G.T = T[m];
        G.passes = gp.passes;
        G.tiles = gp.tiles;
        G.counter_off = off;
        G.team = team;
        G.dl = team > 0 ? sync.dl : 1;
        G.du = team > 0 ? sync.du : 0;
        G.dt = team > 0 ? sync.dt : 0;
        off += gp.tiles;
        out_idx_host[m] = gp.passes % 2;
        const int64_t sh = (gp.geo.nx + 2) * (gp.geo.ny + 2) + (gp.geo.nx + 2) * (gp.geo.nz + 2) +
                           (gp.geo.ny + 2) * (gp.geo.nz + 2);
        h.max_shell = std::max<int64_t>(h.max_shell, sh);
    }
    int it = 0;
    if (team == 0) {
        // within a pass, the grids whose items stream the most planes first
        // (longest processing time first): their next pass, which waits on
        // them, then finds them done more often
        std::vector<int> order(n);
        for (int m = 0; m < n; ++m)
            order[m] = m;
        auto steps = [&](int m) {
            return std::min<int64_t>(plans[m].tp.kchunk, plans[m].geo.nz) + 2 * (int64_t)tl.t;
        };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            return steps(x) != steps(y) ? steps(x) > steps(y) : plans[x].tiles > plans[y].tiles;
        });
        for (int pass = 0; pass < z.maxpasses; ++pass) {
            pass_start[pass] = it;
            for (int m : order) {
                if (pass >= plans[m].passes)
                    continue;
                for (int tile_i = 0; tile_i < plans[m].tiles; ++tile_i)
                    items[it++] = jac::BatchItem{m, pass, tile_i, 0};
            }
        }
    } else {
        const GridPlan &gp = plans[0];
        const int P = gp.passes, nq = gp.tp.nkc, nij = gp.tp.nti * gp.tp.ntj;
        const int lag = sync.dl + 1;
        for (int seg = 0; seg < P; seg += team) {
            const int pe = std::min(P, seg + team);
            for (int64_t w = 0; w < nq + (int64_t)(pe - seg - 1) * lag; ++w)
                for (int pass = seg; pass < pe; ++pass) {
                    const int64_t q = w - (int64_t)(pass - seg) * lag;
                    if (q < 0 || q >= nq)
                        continue;
                    for (int ij = 0; ij < nij; ++ij)
                        items[it++] = jac::BatchItem{0, pass, (int)q * nij + ij, 0};
                }
        }
        // pass ranges do not exist in this order (lockstep runs are refused)
        for (int pass = 0; pass < z.maxpasses; ++pass)
            pass_start[pass] = 0;
    }
    pass_start[z.maxpasses] = it;
    memcpy(img, &h, sizeof h);
    return done(JAC_OK);
}

int jacobi_batched_plan(int dtype, int n, const jac_grid_t *g, void *const *a, void *const *b,
                        const int *T, const jac_tile_t *tile, void *plan_host, size_t plan_bytes,
                        int *out_idx_host)
{
    g_err.clear();
    return build_plan(dtype, n, g, a, b, T, tile, plan_host, plan_bytes, out_idx_host, 0,
                      jac_pipeline_t{1, 0, 0});
}

size_t jacobi_pipelined_plan_bytes(int dtype, const jac_grid_t *g, int T, const jac_tile_t *tile)
{
    g_err.clear();
    jac_tile_t req = tile ? *tile : jac_tile_t{0, 0, 0, 0, 0};
    if (req.kchunk == 0)
        req.kchunk = PIPELINE_KCHUNK;
    return jacobi_batched_plan_bytes(dtype, 1, g, &T, &req);
}

int jacobi_pipelined_plan(int dtype, const jac_grid_t *g, void *a, void *b, int T, int team,
                          const jac_pipeline_t *sync, const jac_tile_t *tile, void *plan_host,
                          size_t plan_bytes, int *out_idx_host)
{
    g_err.clear();
    if (team < 1 || team > 1024)
        return fail(JAC_EARG, "team = %d outside 1..1024", team);
    const jac_pipeline_t sy = sync ? *sync : jac_pipeline_t{1, 0, 0};
    if (sy.dl < 1 || sy.dl > 4096)
        return fail(JAC_EARG, "lower distance dl = %d outside 1..4096", sy.dl);
    if (sy.du != 0 && (sy.du < sy.dl || sy.du > 4096))
        return fail(JAC_EARG, "upper distance du = %d must be 0 (none) or in dl..4096 (dl = %d)", sy.du,
                    sy.dl);
    if (sy.dt < 0 || sy.dt > 4096)
        return fail(JAC_EARG, "team delay dt = %d outside 0..4096", sy.dt);
    jac_tile_t req = tile ? *tile : jac_tile_t{0, 0, 0, 0, 0};
    if (req.kchunk == 0)
        req.kchunk = PIPELINE_KCHUNK;
    void *aa[1] = {a}, *bb[1] = {b};
    return build_plan(dtype, 1, g, aa, bb, &T, &req, plan_host, plan_bytes, out_idx_host, team, sy);
}

// The header of a plan image, checked for the layout the builder writes: the
// grid records, the items and the pass table lie inside the image, and every
// pass range lies inside the item list (a damaged image is refused before
// anything reads past it).
static int read_header(const void *plan_host, jac::BatchHeader *h)
{
    if (!plan_host)
        return fail(JAC_EARG, "plan_host is NULL");
    memcpy(h, plan_host, sizeof *h);
    if (h->magic != jac::BATCH_MAGIC || (h->dtype != JAC_F32 && h->dtype != JAC_F64) || h->n < 1)
        return fail(JAC_EARG, "plan_host is not a batch plan");
    const int64_t total = h->total_bytes;
    const bool layout_ok =
        h->nitems >= 0 && h->ntiles >= 0 && h->maxpasses >= 0 && h->n <= 65535 &&
        h->grids_off >= (int64_t)sizeof(jac::BatchHeader) &&
        h->grids_off + (int64_t)h->n * (int64_t)sizeof(jac::BatchGrid) <= h->items_off &&
        h->items_off + (int64_t)h->nitems * (int64_t)sizeof(jac::BatchItem) <= h->pass_off &&
        h->pass_off + ((int64_t)h->maxpasses + 1) * (int64_t)sizeof(int) <= total;
    if (!layout_ok)
        return fail(JAC_EARG, "plan_host is not a batch plan (damaged layout)");
    const int *pass_start = (const int *)((const unsigned char *)plan_host + h->pass_off);
    if (pass_start[h->maxpasses] != h->nitems)
        return fail(JAC_EARG, "plan_host is not a batch plan (damaged pass table)");
    if (h->order == 0)
        for (int p = 0; p < h->maxpasses; ++p)
            if (pass_start[p] < 0 || pass_start[p] > pass_start[p + 1])
                return fail(JAC_EARG, "plan_host is not a batch plan (damaged pass table)");
    return JAC_OK;
}

// splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): the stress permutation and delays
static uint64_t splitmix64(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int jacobi_batched_stress(void *plan_host, size_t plan_bytes, unsigned seed, int max_delay)
{
    g_err.clear();
    jac::BatchHeader h;
    int rc;
    if ((rc = read_header(plan_host, &h)))
        return rc;
    if ((size_t)h.total_bytes > plan_bytes)
        return fail(JAC_EARG, "plan_bytes = %zu is below the image size %lld", plan_bytes,
                    (long long)h.total_bytes);
    if (max_delay < 0 || max_delay > 64)
        return fail(JAC_EARG, "max_delay = %d outside 0..64", max_delay);
    unsigned char *img = (unsigned char *)plan_host;
    jac::BatchItem *items = (jac::BatchItem *)(img + h.items_off);
    const int *pass_start = (const int *)(img + h.pass_off);
    uint64_t state = seed;
    if (h.order == 0)  // pass-ordered plans: every item waits on earlier passes only
        for (int pass = 0; pass < h.maxpasses; ++pass) {
            const int lo = pass_start[pass], hi = pass_start[pass + 1];
            for (int i = hi - 1; i > lo; --i) {  // Fisher-Yates over [lo, hi)
                const int j = lo + (int)(splitmix64(&state) % (uint64_t)(i - lo + 1));
                std::swap(items[i], items[j]);
            }
        }
    for (int i = 0; i < h.nitems; ++i) {
        const uint64_t r = splitmix64(&state);
        items[i].delay = (max_delay > 0 && r % 4 == 0) ? 1 + (int)((r >> 2) % (uint64_t)max_delay) : 0;
    }
    return JAC_OK;
}

size_t jacobi_batched_workspace(const void *plan_host)
{
    g_err.clear();
    jac::BatchHeader h;
    if (read_header(plan_host, &h))
        return 0;
    return (size_t)(h.ntiles + 2) * sizeof(int);
}

int jacobi_batched_run(const void *plan_host, const void *plan_dev, void *ws, size_t ws_bytes,
                       int mode, void *stream)
{
    g_err.clear();
    jac::BatchHeader h;
    int rc;
    if ((rc = read_header(plan_host, &h)))
        return rc;
    if (!plan_dev || (uintptr_t)plan_dev % 16)
        return fail(JAC_EARG, "plan_dev must be a 16-byte aligned device copy of the plan");
    if (mode != JAC_BATCH_RELAXED && mode != JAC_BATCH_LOCKSTEP)
        return fail(JAC_EARG, "mode must be JAC_BATCH_RELAXED or JAC_BATCH_LOCKSTEP");
    if (h.order != 0 && mode != JAC_BATCH_RELAXED)
        return fail(JAC_EARG, "a pipelined plan runs in relaxed mode only");
    const size_t need = (size_t)(h.ntiles + 2) * sizeof(int);
    if (!ws || ws_bytes < need)
        return fail(JAC_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
    if ((uintptr_t)ws % 4)
        return fail(JAC_EARG, "workspace is not 4-byte aligned");
    if (overlap(ws, need, plan_dev, (size_t)h.total_bytes))
        return fail(JAC_EARG, "workspace overlaps the plan");
    hipStream_t st = (hipStream_t)stream;
    const unsigned char *dimg = (const unsigned char *)plan_dev;
    const jac::BatchGrid *grids = (const jac::BatchGrid *)(dimg + h.grids_off);
    const jac::BatchItem *items = (const jac::BatchItem *)(dimg + h.items_off);
    const int *pass_start = (const int *)((const unsigned char *)plan_host + h.pass_off);
    // every item has the full depth when every grid's T is a multiple of t:
    // then the kernel instance with the depth as a constant runs
    const jac::BatchGrid *hgrids =
        (const jac::BatchGrid *)((const unsigned char *)plan_host + h.grids_off);
    int fixed = 1;
    for (int m = 0; m < h.n; ++m)
        if (hgrids[m].T != hgrids[m].passes * h.t)
            fixed = 0;
    hipError_t e = h.dtype == JAC_F64 ? jac::launch_batch_shells<double>(grids, h.n, h.max_shell, st)
                                      : jac::launch_batch_shells<float>(grids, h.n, h.max_shell, st);
    if (e != hipSuccess)
        return hip_fail(e, "batch shell copy");
    if (h.nitems == 0)
        return JAC_OK;
    jac::BatchLaunch L;
    L.grids = grids;
    L.items = items;
    L.counters = (int *)ws;
    L.error = (int *)ws + h.ntiles + 1;
    L.spin_limit = 1 << 20;
    if (mode == JAC_BATCH_RELAXED) {
        if ((e = jac::launch_zero_ints((int *)ws, h.ntiles + 2, st)) != hipSuccess)
            return hip_fail(e, "counter reset");
        const DeviceFacts dev = device_facts();
        int occ = jac::batched_occupancy(h.dtype, h.cfg, h.t, fixed);
        if (occ < 1)
            occ = 1;
        L.begin = 0;
        L.end = h.nitems;
        L.persistent = 1;
        e = jac::launch_batched(h.dtype, h.cfg, h.t, fixed, L, std::min(h.nitems, dev.cus * occ), st);
        if (e != hipSuccess)
            return hip_fail(e, "batched launch");
    } else {
        for (int pass = 0; pass < h.maxpasses; ++pass) {
            L.begin = pass_start[pass];
            L.end = pass_start[pass + 1];
            L.persistent = 0;
            if (L.end > L.begin &&
                (e = jac::launch_batched(h.dtype, h.cfg, h.t, fixed, L, L.end - L.begin, st)) != hipSuccess)
                return hip_fail(e, "batched pass launch");
        }
    }
    return JAC_OK;
}

int jacobi_autotune(int dtype, const jac_grid_t *g, void *a, void *b, int T, int tmax, int reps,
                    jac_tile_t *best_host, float *best_ms_host, void *stream)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_grid(g, &geo)) ||
        (rc = check_pair(dtype, geo, a, b)))
        return rc;
    if (T < 1)
        return fail(JAC_EARG, "T = %d: autotuning needs T >= 1", T);
    if (tmax < 0 || tmax > JAC_MAX_DEPTH)
        return fail(JAC_EARG, "tmax = %d outside 0..%d", tmax, JAC_MAX_DEPTH);
    if (!best_host)
        return fail(JAC_EARG, "best_host is NULL");
    if (tmax == 0)
        tmax = JAC_MAX_DEPTH;
    if (reps < 1)
        reps = 2;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess)
        return hip_fail(e, "autotune event");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        hipEventDestroy(e0);
        return hip_fail(e, "autotune event");
    }
    const DeviceFacts dev = device_facts();
    float best = 1e30f;
    jac_tile_t pick{0, 0, 0, 0, 0};
    int out = 0;
    for (int n = 0; n < kMenuN; ++n)
        for (int t = 1; t <= std::min(tmax, T); ++t) {
            const jac::TileShape &s = kMenu[n];
            TbPlan probe;
            if (!plan_ij(geo, s, t, &probe) || shape_lds(dtype, s, t) + 1024 > dev.lds_per_block)
                continue;
            // the deepest pass of the split; kernels that spill are skipped
            const int P = (T + t - 1) / t, dmax = T / P + (T % P ? 1 : 0);
            if (jac::tblock_scratch(dtype, s.id, dmax, jac::MODE_PLAIN) != 0)
                continue;
            jac_tile_t cand{t, s.bx(), s.by(), 0, s.waves};
            if ((rc = jacobi_tblock(dtype, g, a, b, T, &cand, nullptr, stream, &out)))
                break;  // warm-up; an error ends the search
            hipEventRecord(e0, st);
            for (int r = 0; r < reps && !rc; ++r)
                rc = jacobi_tblock(dtype, g, a, b, T, &cand, nullptr, stream, &out);
            hipEventRecord(e1, st);
            if ((e = hipEventSynchronize(e1)) != hipSuccess) {
                rc = hip_fail(e, "autotune timing");
                break;
            }
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            ms /= reps;
            if (!rc && ms < best) {
                best = ms;
                pick = cand;
            }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc)
        return rc;
    if (pick.t == 0)
        return fail(JAC_EUNSUPPORTED, "no candidate fits this grid");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_env_tune_once();
        g_tune[TuneKey{device_facts().arch, dtype, geo.nx, geo.ny, geo.nz, geo.sy, geo.sz, T}] =
            TuneEntry{pick, best};
        if (const char *path = tune_env_path())
            if (save_tune_file(path) != JAC_OK)
                fprintf(stderr, "libjacobi: tuning cache not saved: %s\n", g_err.c_str());
    }
    *best_host = pick;
    if (best_ms_host)
        *best_ms_host = best;
    g_err.clear();
    return JAC_OK;
}

int jacobi_tune_save(const char *path)
{
    g_err.clear();
    if (!path || !*path)
        return fail(JAC_EARG, "path is NULL or empty");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_tune_once();
    return save_tune_file(path);
}

int jacobi_tune_load(const char *path, int *n_loaded)
{
    g_err.clear();
    if (!path || !*path)
        return fail(JAC_EARG, "path is NULL or empty");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_tune_once();
    return load_tune_file(path, n_loaded);
}

int jacobi_tune_lookup(const char *arch, int dtype, const jac_grid_t *g, int T, jac_tile_t *tile_host)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_grid(g, &geo)))
        return rc;
    if (!tile_host)
        return fail(JAC_EARG, "tile_host is NULL");
    const std::string a = arch ? std::string(arch) : device_facts().arch;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_tune_once();
    auto it = g_tune.find(TuneKey{a, dtype, geo.nx, geo.ny, geo.nz, geo.sy, geo.sz, T});
    if (it == g_tune.end())
        return fail(JAC_EUNSUPPORTED, "no tuned choice for %s, this geometry and T = %d", a.c_str(), T);
    *tile_host = it->second.tile;
    return JAC_OK;
}

int jacobi_tune_forget(void)
{
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_tune_once();  // so that a later first lookup does not bring the file back
    g_tune.clear();
    return JAC_OK;
}

int jacobi_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    g_err.clear();
    if (!dst || !src)
        return fail(JAC_EARG, "NULL pointer");
    if ((uintptr_t)dst % 16 || (uintptr_t)src % 16 || bytes % 16)
        return fail(JAC_EARG, "pointers and size must be multiples of 16 bytes");
    if (overlap(dst, bytes, src, bytes))
        return fail(JAC_EARG, "ranges overlap");
    if (bytes == 0)
        return JAC_OK;
    hipError_t e = jac::launch_copy(dst, src, bytes, (hipStream_t)stream);
    return e == hipSuccess ? JAC_OK : hip_fail(e, "copy launch");
}

// Checks shared by the lattice Boltzmann entry points (before any HIP call).
static int check_lbm(int dtype, const lbm_grid_t *g, void *f, void *f_tmp, double omega, int T,
                     int *out_idx)
{
    int rc;
    if ((rc = check_dtype(dtype)))
        return rc;
    if (!g)
        return fail(JAC_EARG, "grid descriptor is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(JAC_EARG, "box extents must be >= 1, got %lld x %lld x %lld", (long long)g->nx,
                    (long long)g->ny, (long long)g->nz);
    if (g->nx > (1 << 30) || g->ny > (1 << 30) || g->nz > 65535)
        return fail(JAC_EARG, "box too large (nx, ny <= 2^30, nz <= 65535)");
    const long double cells = (long double)g->nx * g->ny * g->nz;
    if (cells * 19 > (long double)(INT64_MAX / 16) ||
        (long double)((g->nx + 63) / 64) * ((g->ny + 3) / 4) * g->nz > (long double)INT_MAX / 2)
        return fail(JAC_EARG, "box too large");
    if ((rc = check_ptr(f, dtype, "f")) || (rc = check_ptr(f_tmp, dtype, "f_tmp")))
        return rc;
    const int64_t n = g->nx * g->ny * g->nz;
    const size_t bytes = (size_t)(19 * n) * elem_size(dtype);
    if (overlap(f, bytes, f_tmp, bytes))
        return fail(JAC_EARG, "f and f_tmp overlap");
    if (!(omega == omega) || omega > 1e300 || omega < -1e300)
        return fail(JAC_EARG, "omega must be finite");
    if (T < 0)
        return fail(JAC_EARG, "T = %d is negative", T);
    if (!out_idx)
        return fail(JAC_EARG, "out_idx is NULL");
    return JAC_OK;
}

static hipError_t lbm_plain_step(int dtype, const void *src, void *dst, const jac::LbmArgs &p,
                                 hipStream_t st)
{
    return dtype == JAC_F64 ? jac::launch_lbm_d3q19<double>((const double *)src, (double *)dst, p, st)
                            : jac::launch_lbm_d3q19<float>((const float *)src, (float *)dst, p, st);
}

int lbm_d3q19_steps(int dtype, const lbm_grid_t *g, void *f, void *f_tmp, double omega, int T,
                    void *stream, int *out_idx)
{
    g_err.clear();
    int rc;
    if ((rc = check_lbm(dtype, g, f, f_tmp, omega, T, out_idx)))
        return rc;
    *out_idx = 0;
    const int64_t n = g->nx * g->ny * g->nz;
    jac::LbmArgs p{(int)g->nx, (int)g->ny, (int)g->nz, n, omega};
    hipStream_t st = (hipStream_t)stream;
    for (int s = 0; s < T; ++s) {
        void *src = (s % 2 == 0) ? f : f_tmp;
        void *dst = (s % 2 == 0) ? f_tmp : f;
        hipError_t e = lbm_plain_step(dtype, src, dst, p, st);
        if (e != hipSuccess)
            return hip_fail(e, "lattice Boltzmann launch");
    }
    *out_idx = T % 2;
    return JAC_OK;
}

int lbm_d3q19_blocked(int dtype, const lbm_grid_t *g, void *f, void *f_tmp, double omega, int T,
                      int kchunk, void *stream, int *out_idx)
{
    g_err.clear();
    int rc;
    if ((rc = check_lbm(dtype, g, f, f_tmp, omega, T, out_idx)))
        return rc;
    if (kchunk < 0 || kchunk > 65535)
        return fail(JAC_EARG, "kchunk = %d outside 0..65535", kchunk);
    // default z chunk, measured at 256^3 on MI355X: short chunks keep the
    // workgroups that run together on the same few planes, whose halo planes
    // the neighbouring chunks then find in L2 (FP64 20.9 GLUP/s at 12 planes
    // against 17.2 at 64; FP32 37.6 at 4 against 29.8)
    const int def_kc = dtype == JAC_F64 ? 12 : 4;
    const int kc = (int)std::min<int64_t>(kchunk ? kchunk : def_kc, g->nz);
    const int rx = jac::lbm2_region_x(elem_size(dtype)), ry = jac::lbm2_region_y(elem_size(dtype));
    const int64_t gx = (g->nx + rx - 3) / (rx - 2);
    const int64_t gy = (g->ny + ry - 3) / (ry - 2);
    const int64_t gz = (g->nz + kc - 1) / kc;
    if (gy > 65535 || (long double)gx * gy * gz > (long double)INT_MAX / 2)
        return fail(JAC_EARG, "box too large for the two-step pass (ceil(ny/%d) <= 65535)", ry - 2);
    *out_idx = 0;
    const int64_t n = g->nx * g->ny * g->nz;
    jac::LbmArgs p{(int)g->nx, (int)g->ny, (int)g->nz, n, omega};
    hipStream_t st = (hipStream_t)stream;
    int launches = 0;
    for (int s = 0; s < T; launches++) {
        void *src = (launches % 2 == 0) ? f : f_tmp;
        void *dst = (launches % 2 == 0) ? f_tmp : f;
        hipError_t e;
        if (T - s >= 2) {
            e = dtype == JAC_F64 ? jac::launch_lbm_d3q19_x2<double>((const double *)src, (double *)dst, p,
                                                                     kc, st)
                                 : jac::launch_lbm_d3q19_x2<float>((const float *)src, (float *)dst, p,
                                                                    kc, st);
            s += 2;
        } else {
            e = lbm_plain_step(dtype, src, dst, p, st);
            s += 1;
        }
        if (e != hipSuccess)
            return hip_fail(e, "lattice Boltzmann launch");
    }
    *out_idx = launches % 2;
    return JAC_OK;
}

int jacobi_tile_menu(int dtype, int *shapes_host, int cap)
{
    g_err.clear();
    if (check_dtype(dtype))
        return JAC_EARG;
    if (cap < 0 || (cap > 0 && !shapes_host))
        return fail(JAC_EARG, "bad output array");
    for (int n = 0; n < kMenuN && n < cap; ++n) {
        shapes_host[3 * n] = kMenu[n].bx();
        shapes_host[3 * n + 1] = kMenu[n].by();
        shapes_host[3 * n + 2] = kMenu[n].waves;
    }
    return kMenuN;
}

int jacobi_default_tile(int dtype, const jac_grid_t *g, int T, int t, int kind, jac_tile_t *tile_host)
{
    g_err.clear();
    Geo geo;
    int rc;
    if ((rc = check_dtype(dtype)) || (rc = check_grid(g, &geo)))
        return rc;
    if (!tile_host)
        return fail(JAC_EARG, "tile_host is NULL");
    if (T < 0)
        return fail(JAC_EARG, "T = %d is negative", T);
    if (kind < 0 || kind > 2)
        return fail(JAC_EARG, "kind = %d is not 0 (plain), 1 (right-hand side) or 2 (adjoint)",
                    kind);
    // the same resolution as jacobi_tblock and jacobi_adjoint: only the plain
    // pass consults the tuning cache, which is keyed by its geometry
    const int k = kind == 2 ? KIND_TRACE : kind == 1 ? KIND_RHS : KIND_PLAIN;
    jac_tile_t req{t, 0, 0, 0, 0};
    if ((rc = resolve_tile(dtype, &req, T, tile_host, k == KIND_PLAIN ? &geo : nullptr, k)))
        return rc;
    return JAC_OK;
}

}  // extern "C"
