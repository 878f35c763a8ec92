// z4c_api.hip -- host side of libz4c.so: the C ABI declared in include/z4c.h.
//
// Every argument is validated here, before anything is enqueued, so invalid
// calls are testable without a GPU.  The kernels receive the box geometry by
// value (BoxSet), so the single-box entry points allocate nothing and the
// batched plan needs no device-side tables either.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "z4c_internal.h"

using namespace z4c;

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string& msg)
{
    g_last_error = msg;
    return status;
}

int hip_fail(hipError_t e, const char* where)
{
    return fail(Z4C_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

std::mutex g_tile_mu;
int g_selected[2] = {-1, -1};   // per precision: index into the tile table, -1 = default
int g_selected_pers[2] = {0, 0};

int default_tile_index(int precision, int* persistent = nullptr)
{
    const TileEntry* t = nullptr;
    const int n = tile_table(&t);
    if (persistent) *persistent = 0;
    {
        std::lock_guard<std::mutex> lk(g_tile_mu);
        if (g_selected[precision] >= 0) {
            if (persistent) *persistent = g_selected_pers[precision];
            return g_selected[precision];
        }
    }
    // the shape measured fastest on large boxes (8x8x8 bricks, two waves per
    // SIMD) when compiled, else the first of the precision
    for (int i = 0; i < n; ++i)
        if (t[i].precision == precision && t[i].tile.bx == 8 && t[i].tile.by == 8 && t[i].tile.bz == 8 &&
            t[i].tile.waves == 2)
            return i;
    for (int i = 0; i < n; ++i)
        if (t[i].precision == precision) return i;
    return -1;
}

int find_tile(int precision, const z4c_tile* want)
{
    const TileEntry* t = nullptr;
    const int n = tile_table(&t);
    for (int i = 0; i < n; ++i)
        if (t[i].precision == precision && t[i].tile.bx == want->bx && t[i].tile.by == want->by &&
            t[i].tile.bz == want->bz && t[i].tile.waves == want->waves)
            return i;
    return -1;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int check_params(const z4c_params* p)
{
    if (!p) return fail(Z4C_EINVAL, "params is NULL");
    if (p->precision != Z4C_FP64 && p->precision != Z4C_MIXED)
        return fail(Z4C_EINVAL, "unknown precision " + std::to_string(p->precision));
    const double v[] = {p->kappa1, p->kappa2, p->kappa3, p->eta, p->shift_coeff, p->ko_sigma, p->w_floor};
    for (double x : v)
        if (!std::isfinite(x)) return fail(Z4C_EINVAL, "non-finite parameter");
    if (!(p->w_floor > 0.0)) return fail(Z4C_EINVAL, "w_floor must be > 0");
    if (p->ko_sigma < 0.0) return fail(Z4C_EINVAL, "ko_sigma must be >= 0");
    return Z4C_OK;
}

ParamsDev to_dev(const z4c_params* p)
{
    return ParamsDev{p->kappa1, p->kappa2, p->kappa3, p->eta, p->shift_coeff, p->ko_sigma, p->w_floor,
                     p->lapse_uses_K ? 1 : 0};
}

// Geometry checks shared by every entry point.  On success fills the
// stored extent (points per field).
int check_geom(long sf, int nx, int ny, int nz, int ng, int bc, long* stored)
{
    if (nx < 1 || ny < 1 || nz < 1) return fail(Z4C_EINVAL, "active extents must be >= 1");
    if (ng < 3) return fail(Z4C_EINVAL, "ghost width ng must be >= 3 (stencil reach)");
    if (bc < Z4C_BC_PERIODIC || bc > Z4C_BC_EQUATORIAL) return fail(Z4C_EINVAL, "unknown boundary kind");
    const long Nx = (long)nx + 2L * ng, Ny = (long)ny + 2L * ng, Nz = (long)nz + 2L * ng;
    if (Nx > (1L << 20) || Ny > (1L << 20) || Nz > (1L << 20)) return fail(Z4C_EINVAL, "extent too large");
    const long n = Nx * Ny * Nz;
    if (n > (1L << 31) - 1) return fail(Z4C_EINVAL, "more than 2^31-1 stored points per field");
    if (sf < n) return fail(Z4C_EINVAL, "field stride sf is smaller than the stored points per field");
    if (sf > (INT64_MAX / 8) / NF) return fail(Z4C_EINVAL, "field stride too large");
    *stored = n;
    return Z4C_OK;
}

int check_spacing(double dx, double dy, double dz, double x0, double y0, double z0)
{
    if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(dz)) return fail(Z4C_EINVAL, "spacings must be finite and > 0");
    if (!std::isfinite(x0) || !std::isfinite(y0) || !std::isfinite(z0)) return fail(Z4C_EINVAL, "non-finite origin");
    return Z4C_OK;
}

bool overlap(const void* a, const void* b, long sf)
{
    if (!a || !b) return false;
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b, len = (uintptr_t)sf * NF * sizeof(double);
    return pa < pb + len && pb < pa + len;
}

// two state arrays of different field strides
bool overlap2(const void* a, long sfa, const void* b, long sfb)
{
    if (!a || !b) return false;
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    const uintptr_t la = (uintptr_t)sfa * NF * sizeof(double), lb = (uintptr_t)sfb * NF * sizeof(double);
    return pa < pb + lb && pb < pa + la;
}

long bricks(const int n[3], const z4c_tile& t, int nb[3])
{
    nb[0] = (n[0] + t.bx - 1) / t.bx;
    nb[1] = (n[1] + t.by - 1) / t.by;
    nb[2] = (n[2] + t.bz - 1) / t.bz;
    return (long)nb[0] * nb[1] * nb[2];
}

long shell_size(const int n[3], int ng)
{
    const long N0 = n[0] + 2L * ng, N1 = n[1] + 2L * ng, N2 = n[2] + 2L * ng;
    return N0 * N1 * N2 - (long)n[0] * n[1] * n[2];
}

BoxDev make_box(const int n[3], int ng, int bc, long sf, const double h[3], const double x0[3], double dt)
{
    BoxDev b{};
    b.sf = sf;
    for (int d = 0; d < 3; ++d) {
        b.n[d] = n[d];
        b.h[d] = h[d];
        b.x0[d] = x0[d];
    }
    b.ng = ng;
    b.bc = bc;
    b.dt = dt;
    return b;
}

// fill the prefix sums of a set for the given tile
void finalize_set(BoxSet& s, const z4c_tile& t)
{
    s.brick_begin[0] = 0;
    s.shell_begin[0] = 0;
    for (int b = 0; b < s.nbox; ++b) {
        s.brick_begin[b + 1] = s.brick_begin[b] + bricks(s.box[b].n, t, s.box[b].nb);
        s.shell_begin[b + 1] = s.shell_begin[b] + shell_size(s.box[b].n, s.box[b].ng);
    }
}

// ---------------------------------------------------------------------------
// Persisted tile tuning.  The cache is a text file of JSON lines, one object
// per (device architecture, precision, box count, workload bucket):
//   {"arch": "gfx950", "precision": 0, "nbox": 1, "bucket": 24, "tile": [8, 8, 8, 2, 1], "ms": 29.4}
// bucket = floor(log2(total active cells)).  Reading is strict: any line that
// is not such an object makes the whole file corrupt (Z4C_EINVAL), so that a
// damaged cache is reported instead of silently ignored.
// ---------------------------------------------------------------------------
struct TuneEntry {
    std::string arch;
    int precision = -1, nbox = -1, bucket = -1;
    z4c_tile tile{};
    double ms = 0.0;
};

struct LineParser {
    const char* p;
    void ws()
    {
        while (*p == ' ' || *p == '\t' || *p == '\r') ++p;
    }
    bool lit(char c)
    {
        ws();
        if (*p != c) return false;
        ++p;
        return true;
    }
    bool str(std::string& out)
    {
        ws();
        if (*p != '"') return false;
        ++p;
        out.clear();
        while (*p && *p != '"') {
            const char c = *p++;
            const bool ok = (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || (c >= '0' && c <= '9') || c == '_' ||
                            c == '-' || c == '+' || c == ':' || c == '.';
            if (!ok || out.size() > 64) return false;
            out.push_back(c);
        }
        if (*p != '"') return false;
        ++p;
        return true;
    }
    bool integer(int& v)
    {
        ws();
        char* e = nullptr;
        const long x = std::strtol(p, &e, 10);
        if (e == p || x < -1000000 || x > 1000000) return false;
        p = e;
        v = (int)x;
        return true;
    }
    bool number(double& v)
    {
        ws();
        char* e = nullptr;
        v = std::strtod(p, &e);
        if (e == p || !std::isfinite(v)) return false;
        p = e;
        return true;
    }
};

// parse one line into e; false if it is not a complete entry
bool tune_parse_line(const char* line, TuneEntry& e)
{
    LineParser L{line};
    if (!L.lit('{')) return false;
    bool has_arch = false, has_prec = false, has_nbox = false, has_bucket = false, has_tile = false;
    for (bool first = true;; first = false) {
        if (L.lit('}')) break;
        if (!first && !L.lit(',')) return false;
        std::string key;
        if (!L.str(key) || !L.lit(':')) return false;
        if (key == "arch" && !has_arch) {
            if (!(has_arch = L.str(e.arch))) return false;
        } else if (key == "precision" && !has_prec) {
            if (!(has_prec = L.integer(e.precision))) return false;
        } else if (key == "nbox" && !has_nbox) {
            if (!(has_nbox = L.integer(e.nbox))) return false;
        } else if (key == "bucket" && !has_bucket) {
            if (!(has_bucket = L.integer(e.bucket))) return false;
        } else if (key == "ms") {
            if (!L.number(e.ms)) return false;
        } else if (key == "tile" && !has_tile) {
            int v[5];
            if (!L.lit('[')) return false;
            for (int i = 0; i < 5; ++i)
                if ((i > 0 && !L.lit(',')) || !L.integer(v[i])) return false;
            if (!L.lit(']')) return false;
            e.tile = z4c_tile{v[0], v[1], v[2], v[3], v[4]};
            has_tile = true;
        } else
            return false;
    }
    L.ws();
    if (*L.p != '\0' && *L.p != '\n') return false;
    return has_arch && has_prec && has_nbox && has_bucket && has_tile && !e.arch.empty() &&
           (e.precision == Z4C_FP64 || e.precision == Z4C_MIXED) && e.nbox >= 1 && e.nbox <= MAXBOX &&
           e.bucket >= 0 && e.bucket < 64 && (e.tile.persistent == 0 || e.tile.persistent == 1);
}

// Read every entry of the cache.  A missing file is an empty cache.
int tune_read(const char* path, std::vector<TuneEntry>& out)
{
    out.clear();
    FILE* f = std::fopen(path, "r");
    if (!f) return Z4C_OK;
    char line[1024];
    int no = 0;
    while (std::fgets(line, sizeof line, f)) {
        ++no;
        const size_t len = std::strlen(line);
        if (len + 1 == sizeof line && line[len - 1] != '\n') {
            std::fclose(f);
            return fail(Z4C_EINVAL, std::string("tune cache ") + path + ": line " + std::to_string(no) + " too long");
        }
        const char* q = line;
        while (*q == ' ' || *q == '\t' || *q == '\r' || *q == '\n') ++q;
        if (*q == '\0') continue;  // blank line
        TuneEntry e;
        if (!tune_parse_line(line, e)) {
            std::fclose(f);
            return fail(Z4C_EINVAL, std::string("tune cache ") + path + ": line " + std::to_string(no) +
                                        " is not a tuning entry");
        }
        out.push_back(e);
    }
    std::fclose(f);
    return Z4C_OK;
}

const TuneEntry* tune_find(const std::vector<TuneEntry>& v, const std::string& arch, int precision, int nbox,
                           int bucket)
{
    for (const TuneEntry& e : v)
        if (e.arch == arch && e.precision == precision && e.nbox == nbox && e.bucket == bucket) return &e;
    return nullptr;
}

// Replace (or add) the entry of e's key and rewrite the file atomically.
int tune_write(const char* path, const TuneEntry& e)
{
    std::vector<TuneEntry> v;
    int rc = tune_read(path, v);
    if (rc) return rc;
    bool done = false;
    for (TuneEntry& x : v)
        if (x.arch == e.arch && x.precision == e.precision && x.nbox == e.nbox && x.bucket == e.bucket) {
            x = e;
            done = true;
        }
    if (!done) v.push_back(e);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return fail(Z4C_EINVAL, "cannot write tune cache " + tmp);
    for (const TuneEntry& x : v)
        std::fprintf(f, "{\"arch\": \"%s\", \"precision\": %d, \"nbox\": %d, \"bucket\": %d, "
                        "\"tile\": [%d, %d, %d, %d, %d], \"ms\": %.4f}\n",
                     x.arch.c_str(), x.precision, x.nbox, x.bucket, x.tile.bx, x.tile.by, x.tile.bz, x.tile.waves,
                     x.tile.persistent, x.ms);
    const bool ok = std::fflush(f) == 0;
    std::fclose(f);
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(Z4C_EINVAL, std::string("cannot write tune cache ") + path);
    }
    return Z4C_OK;
}

// architecture name of the current device without feature suffixes ("gfx950")
int device_arch(std::string& arch)
{
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "device architecture query");
    arch = prop.gcnArchName;
    const size_t c = arch.find(':');
    if (c != std::string::npos) arch.resize(c);
    return Z4C_OK;
}

int cells_bucket(const z4c_box* boxes, int nbox)
{
    double cells = 0.0;
    for (int b = 0; b < nbox; ++b) cells += (double)boxes[b].n[0] * boxes[b].n[1] * boxes[b].n[2];
    int k = 0;
    while (k < 62 && std::ldexp(1.0, k + 1) <= cells) ++k;
    return k;
}

}  // namespace

extern "C" {

void z4c_default_params(z4c_params* p)
{
    if (!p) return;
    p->kappa1 = 0.005;
    p->kappa2 = 0.0;
    p->kappa3 = 0.0;
    p->eta = 0.36;
    p->shift_coeff = 0.75;
    p->ko_sigma = 0.5;
    p->w_floor = 1e-10;
    p->lapse_uses_K = 0;
    p->precision = Z4C_FP64;
}

const char* z4c_strerror(int status)
{
    switch (status) {
    case Z4C_OK: return "ok";
    case Z4C_EINVAL: return "invalid argument";
    case Z4C_EHIP: return "HIP runtime error";
    case Z4C_ENOMEM: return "out of memory";
    case Z4C_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

const char* z4c_last_error(void) { return g_last_error.c_str(); }

int z4c_tile_count(int precision)
{
    const TileEntry* t = nullptr;
    const int n = tile_table(&t);
    int c = 0;
    for (int i = 0; i < n; ++i) c += t[i].precision == precision;
    return c;
}

int z4c_tile_get(int precision, int index, z4c_tile* out)
{
    if (!out) return fail(Z4C_EINVAL, "out is NULL");
    const TileEntry* t = nullptr;
    const int n = tile_table(&t);
    int c = 0;
    for (int i = 0; i < n; ++i) {
        if (t[i].precision != precision) continue;
        if (c++ == index) {
            *out = t[i].tile;
            return Z4C_OK;
        }
    }
    return fail(Z4C_EINVAL, "tile index out of range");
}

int z4c_select_tile(int precision, const z4c_tile* tile)
{
    if (precision != Z4C_FP64 && precision != Z4C_MIXED) return fail(Z4C_EINVAL, "unknown precision");
    int idx = -1;
    if (tile) {
        idx = find_tile(precision, tile);
        if (idx < 0) return fail(Z4C_EUNSUPPORTED, "no compiled tile of that shape");
    }
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_selected[precision] = idx;
    g_selected_pers[precision] = (tile && tile->persistent) ? 1 : 0;
    return Z4C_OK;
}

int z4c_tile_resources(int precision, const z4c_tile* tile, int* waves_per_simd, int* lds_bytes, int* scratch_bytes)
{
    if (precision != Z4C_FP64 && precision != Z4C_MIXED) return fail(Z4C_EINVAL, "unknown precision");
    if (!tile || !waves_per_simd || !lds_bytes || !scratch_bytes)
        return fail(Z4C_EINVAL, "tile and the three outputs must be non-NULL");
    const int idx = find_tile(precision, tile);
    if (idx < 0) return fail(Z4C_EUNSUPPORTED, "no compiled tile of that shape");
    const TileEntry* t = nullptr;
    tile_table(&t);
    const hipError_t e = t[idx].resources(waves_per_simd, lds_bytes, scratch_bytes);
    if (e != hipSuccess) return hip_fail(e, "kernel attribute query");
    return Z4C_OK;
}

int rhs_z4c(const double* u, double* rhs, long sf, int nx, int ny, int nz, int ng, double dx, double dy, double dz,
            double x0, double y0, double z0, int bc, const z4c_params* p, void* stream)
{
    long stored = 0;
    int rc;
    if ((rc = check_params(p)) || (rc = check_geom(sf, nx, ny, nz, ng, bc, &stored)) ||
        (rc = check_spacing(dx, dy, dz, x0, y0, z0)))
        return rc;
    if (!u || !rhs) return fail(Z4C_EINVAL, "u and rhs must be non-NULL");
    if (overlap(u, rhs, sf)) return fail(Z4C_EINVAL, "u and rhs overlap");
    int pers = 0;
    const int ti = default_tile_index(p->precision, &pers);
    if (ti < 0) return fail(Z4C_EUNSUPPORTED, "no tile compiled for this precision");
    const TileEntry* tab = nullptr;
    tile_table(&tab);
    const int n[3] = {nx, ny, nz};
    const double h[3] = {dx, dy, dz}, o[3] = {x0, y0, z0};
    BoxSet set{};
    set.nbox = 1;
    set.box[0] = make_box(n, ng, bc, sf, h, o, 1.0);
    set.box[0].u_in = u;
    set.box[0].u_out = rhs;
    finalize_set(set, tab[ti].tile);
    const ParamsDev pd = to_dev(p);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pending HIP error before rhs_z4c");
    if ((e = tab[ti].launch(set, pd, MODE_RHS, 0, pers, s)) != hipSuccess)
        return hip_fail(e, "rhs_z4c fused launch");
    if ((e = launch_sommerfeld(set, pd, MODE_RHS, 0, s)) != hipSuccess) return hip_fail(e, "rhs_z4c ghost launch");
    return Z4C_OK;
}

int rk4_substep(int stage, double dt, const double* u_in, const double* u_n, double* acc, double* u_out, long sf,
                int nx, int ny, int nz, int ng, double dx, double dy, double dz, double x0, double y0, double z0,
                int bc, const z4c_params* p, void* stream)
{
    long stored = 0;
    int rc;
    if ((rc = check_params(p)) || (rc = check_geom(sf, nx, ny, nz, ng, bc, &stored)) ||
        (rc = check_spacing(dx, dy, dz, x0, y0, z0)))
        return rc;
    if (stage < 1 || stage > 4) return fail(Z4C_EINVAL, "stage must be 1..4");
    if (!finite_pos(dt)) return fail(Z4C_EINVAL, "dt must be finite and > 0");
    if (!u_in || !acc || !u_out) return fail(Z4C_EINVAL, "u_in, acc and u_out must be non-NULL");
    if ((stage == 2 || stage == 3) && !u_n) return fail(Z4C_EINVAL, "stages 2 and 3 read u_n");
    if (overlap(u_out, u_in, sf)) return fail(Z4C_EINVAL, "u_out overlaps u_in");
    if (overlap(u_out, acc, sf)) return fail(Z4C_EINVAL, "u_out overlaps acc");
    if (overlap(acc, u_in, sf)) return fail(Z4C_EINVAL, "acc overlaps u_in");
    if (stage != 4 && stage != 1 && overlap(acc, u_n, sf)) return fail(Z4C_EINVAL, "acc overlaps u_n");
    if ((stage == 2 || stage == 3) && overlap(u_out, u_n, sf))
        return fail(Z4C_EINVAL, "u_out may alias u_n only in stage 4");
    int pers = 0;
    const int ti = default_tile_index(p->precision, &pers);
    if (ti < 0) return fail(Z4C_EUNSUPPORTED, "no tile compiled for this precision");
    const TileEntry* tab = nullptr;
    tile_table(&tab);
    const int n[3] = {nx, ny, nz};
    const double h[3] = {dx, dy, dz}, o[3] = {x0, y0, z0};
    BoxSet set{};
    set.nbox = 1;
    set.box[0] = make_box(n, ng, bc, sf, h, o, dt);
    set.box[0].u_in = u_in;
    set.box[0].u_n = u_n;
    set.box[0].acc = acc;
    set.box[0].u_out = u_out;
    finalize_set(set, tab[ti].tile);
    const ParamsDev pd = to_dev(p);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pending HIP error before rk4_substep");
    if ((e = tab[ti].launch(set, pd, MODE_STAGE, stage, pers, s)) != hipSuccess)
        return hip_fail(e, "rk4_substep fused launch");
    if ((bc == Z4C_BC_SOMMERFELD || bc == Z4C_BC_EQUATORIAL) &&
        (e = launch_sommerfeld(set, pd, MODE_STAGE, stage, s)) != hipSuccess)
        return hip_fail(e, "rk4_substep Sommerfeld launch");
    return Z4C_OK;
}

long z4c_monitor_workspace(int nx, int ny, int nz)
{
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    const int n[3] = {nx, ny, nz};
    return monitor_records_max(n) * 4;
}

int rk4_substep_monitor(int stage, double dt, const double* u_in, const double* u_n, double* acc, double* u_out,
                        long sf, int nx, int ny, int nz, int ng, double dx, double dy, double dz, double x0, double y0,
                        double z0, int bc, const z4c_params* p, double* c, double* norms, double* ws, long ws_len,
                        void* stream)
{
    long stored = 0;
    int rc;
    if ((rc = check_params(p)) || (rc = check_geom(sf, nx, ny, nz, ng, bc, &stored)) ||
        (rc = check_spacing(dx, dy, dz, x0, y0, z0)))
        return rc;
    if (p->precision != Z4C_FP64) return fail(Z4C_EUNSUPPORTED, "the stage monitor runs in float64 only");
    if (stage < 1 || stage > 4) return fail(Z4C_EINVAL, "stage must be 1..4");
    if (!finite_pos(dt)) return fail(Z4C_EINVAL, "dt must be finite and > 0");
    if (!u_in || !acc || !u_out) return fail(Z4C_EINVAL, "u_in, acc and u_out must be non-NULL");
    if (!norms || !ws) return fail(Z4C_EINVAL, "norms and ws must be non-NULL");
    if ((stage == 2 || stage == 3) && !u_n) return fail(Z4C_EINVAL, "stages 2 and 3 read u_n");
    if (overlap(u_out, u_in, sf)) return fail(Z4C_EINVAL, "u_out overlaps u_in");
    if (overlap(u_out, acc, sf)) return fail(Z4C_EINVAL, "u_out overlaps acc");
    if (overlap(acc, u_in, sf)) return fail(Z4C_EINVAL, "acc overlaps u_in");
    if (stage != 4 && stage != 1 && overlap(acc, u_n, sf)) return fail(Z4C_EINVAL, "acc overlaps u_n");
    if ((stage == 2 || stage == 3) && overlap(u_out, u_n, sf))
        return fail(Z4C_EINVAL, "u_out may alias u_n only in stage 4");
    const long need = z4c_monitor_workspace(nx, ny, nz);
    if (ws_len < need) return fail(Z4C_EINVAL, "workspace too small: need " + std::to_string(need) + " doubles");
    // c (4 fields), ws and norms against every state array and each other
    const void* states[4] = {u_in, u_n, acc, u_out};
    for (const void* a : states) {
        if (c && overlap2(c, sf * 4 / NF + 1, a, sf)) return fail(Z4C_EINVAL, "c overlaps a state array");
        if (overlap2(ws, need / NF + 1, a, sf)) return fail(Z4C_EINVAL, "ws overlaps a state array");
        if (overlap2(norms, 1, a, sf)) return fail(Z4C_EINVAL, "norms overlaps a state array");
    }
    if (c && (overlap2(c, sf * 4 / NF + 1, ws, need / NF + 1) || overlap2(c, sf * 4 / NF + 1, norms, 1)))
        return fail(Z4C_EINVAL, "c overlaps ws or norms");
    if (overlap2(ws, need / NF + 1, norms, 1)) return fail(Z4C_EINVAL, "ws overlaps norms");
    const int n[3] = {nx, ny, nz};
    const double h[3] = {dx, dy, dz}, o[3] = {x0, y0, z0};
    BoxSet set{};
    set.nbox = 1;
    set.box[0] = make_box(n, ng, bc, sf, h, o, dt);
    set.box[0].u_in = u_in;
    set.box[0].u_n = u_n;
    set.box[0].acc = acc;
    set.box[0].u_out = u_out;
    finalize_set(set, z4c_tile{8, 8, 8, 2, 1});
    const ParamsDev pd = to_dev(p);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pending HIP error before rk4_substep_monitor");
    if (c && (e = launch_zero(c, 4 * sf, s)) != hipSuccess) return hip_fail(e, "rk4_substep_monitor zero fill");
    long records = 0;
    if ((e = launch_stage_monitor(set, pd, MODE_STAGE, stage, MonDev{c, ws}, s, &records)) != hipSuccess)
        return hip_fail(e, "rk4_substep_monitor fused launch");
    if ((bc == Z4C_BC_SOMMERFELD || bc == Z4C_BC_EQUATORIAL) &&
        (e = launch_sommerfeld(set, pd, MODE_STAGE, stage, s)) != hipSuccess)
        return hip_fail(e, "rk4_substep_monitor Sommerfeld launch");
    if ((e = launch_norms(ws, records, 1.0 / ((double)nx * ny * nz), norms, s)) != hipSuccess)
        return hip_fail(e, "rk4_substep_monitor norms");
    return Z4C_OK;
}

int apply_ghosts(double* u, const double* shell, long sf, int nx, int ny, int nz, int ng, int bc, void* stream)
{
    long stored = 0;
    int rc;
    if ((rc = check_geom(sf, nx, ny, nz, ng, bc, &stored))) return rc;
    if (!u) return fail(Z4C_EINVAL, "u is NULL");
    if (bc == Z4C_BC_COPY && !shell) return fail(Z4C_EINVAL, "a copy box needs its ghost shell");
    if (bc != Z4C_BC_COPY && shell) return fail(Z4C_EINVAL, "shell must be NULL unless bc is Z4C_BC_COPY");
    if (bc == Z4C_BC_SOMMERFELD) return Z4C_OK;
    const int n[3] = {nx, ny, nz};
    const long ns = shell_size(n, ng);
    if (shell) {
        const uintptr_t a = (uintptr_t)u, b = (uintptr_t)shell;
        const uintptr_t la = (uintptr_t)sf * NF * 8, lb = (uintptr_t)ns * NF * 8;
        if (a < b + lb && b < a + la) return fail(Z4C_EINVAL, "shell overlaps u");
    }
    const double h[3] = {1, 1, 1}, o[3] = {0, 0, 0};
    BoxSet set{};
    set.nbox = 1;
    set.box[0] = make_box(n, ng, bc, sf, h, o, 1.0);
    set.box[0].u_in = u;
    set.box[0].shell = shell;
    z4c_tile t{8, 8, 4, 1, 0};
    finalize_set(set, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pending HIP error before apply_ghosts");
    if ((e = launch_ghosts(set, (hipStream_t)stream)) != hipSuccess) return hip_fail(e, "apply_ghosts launch");
    return Z4C_OK;
}

long z4c_constraints_workspace(int nx, int ny, int nz)
{
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    const int n[3] = {nx, ny, nz};
    return 4 * constraint_blocks(n);
}

// Validation and launch shared by z4c_constraints and z4c_constraints_noalloc;
// ws is the caller's workspace, or the library's fixed device array (whose
// overlap with the arguments needs no check: no caller can hold it).
static int constraints_impl(const double* u, double* c, double* norms, double* ws, bool own_ws, long sf, int nx,
                            int ny, int nz, int ng, double dx, double dy, double dz, void* stream, const char* where)
{
    auto span = [](const void* p, uintptr_t bytes, const void* q, uintptr_t qbytes) {
        const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
        return a < b + qbytes && b < a + bytes;
    };
    const long need = z4c_constraints_workspace(nx, ny, nz);
    const uintptr_t ub = (uintptr_t)sf * NF * 8, cb = (uintptr_t)sf * 4 * 8, wb = (uintptr_t)need * 8;
    if (c && span(c, cb, u, ub)) return fail(Z4C_EINVAL, "c overlaps u");
    if (!own_ws && (span(ws, wb, u, ub) || (c && span(ws, wb, c, cb)) || span(ws, wb, norms, 32)))
        return fail(Z4C_EINVAL, "ws overlaps another argument");
    if (span(norms, 32, u, ub) || (c && span(norms, 32, c, cb))) return fail(Z4C_EINVAL, "norms overlaps another argument");
    const int n[3] = {nx, ny, nz};
    const double h[3] = {dx, dy, dz}, o[3] = {0, 0, 0};
    BoxSet set{};
    set.nbox = 1;
    set.box[0] = make_box(n, ng, Z4C_BC_PERIODIC, sf, h, o, 1.0);
    set.box[0].u_in = u;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, (std::string("pending HIP error before ") + where).c_str());
    if ((e = launch_constraints(set, c, norms, ws, (hipStream_t)stream)) != hipSuccess)
        return hip_fail(e, (std::string(where) + " launch").c_str());
    return Z4C_OK;
}

int z4c_constraints(const double* u, double* c, double* norms, double* ws, long ws_len, long sf, int nx, int ny,
                    int nz, int ng, double dx, double dy, double dz, void* stream)
{
    long stored = 0;
    int rc;
    if ((rc = check_geom(sf, nx, ny, nz, ng, Z4C_BC_PERIODIC, &stored)) ||
        (rc = check_spacing(dx, dy, dz, 0.0, 0.0, 0.0)))
        return rc;
    if (!u || !norms || !ws) return fail(Z4C_EINVAL, "u, norms and ws must be non-NULL");
    const long need = z4c_constraints_workspace(nx, ny, nz);
    if (ws_len < need) return fail(Z4C_EINVAL, "workspace too small: need " + std::to_string(need) + " doubles");
    return constraints_impl(u, c, norms, ws, false, sf, nx, ny, nz, ng, dx, dy, dz, stream, "z4c_constraints");
}

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------
struct z4c_plan_s {
    std::vector<z4c_box> boxes;
    ParamsDev prm;
    int precision;
    int tile_index;
    int persistent;    // grid capped at the resident-block count, bricks walked in a loop
    int tile_source;   // Z4C_TILE_DEFAULT / CALLER / CACHE / TUNED
    BoxSet fused[4];   // per stage
    BoxSet ghosts[4];  // per stage: fill of the stage input
    bool any_ghost_fill, any_sommerfeld;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t capture;  // private stream the step is captured on (never the legacy stream)
};

static void plan_build_sets(z4c_plan_s* P)
{
    const TileEntry* tab = nullptr;
    tile_table(&tab);
    const z4c_tile& t = tab[P->tile_index].tile;
    for (int s = 0; s < 4; ++s) {
        BoxSet& F = P->fused[s];
        BoxSet& G = P->ghosts[s];
        F = BoxSet{};
        G = BoxSet{};
        F.nbox = G.nbox = (int)P->boxes.size();
        for (int b = 0; b < F.nbox; ++b) {
            const z4c_box& x = P->boxes[b];
            BoxDev d = make_box(x.n, x.ng, x.bc, x.sf, x.dx, x.x0, x.dt);
            const double* in = s == 0 ? x.u_n : (s == 2 ? x.u_b : x.u_a);
            double* out = s == 0 ? x.u_a : (s == 1 ? x.u_b : (s == 2 ? x.u_a : x.u_n));
            d.u_in = in;
            d.u_n = x.u_n;
            d.acc = x.acc;
            d.u_out = out;
            d.shell = x.shell;
            F.box[b] = d;
            G.box[b] = d;
        }
        finalize_set(F, t);
        finalize_set(G, t);
    }
}

static void plan_drop_graph(z4c_plan_s* P)
{
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    P->exec = nullptr;
    P->graph = nullptr;
}

// enqueue one RK4 step of every box
static hipError_t plan_enqueue_step(z4c_plan_s* P, hipStream_t s)
{
    const TileEntry* tab = nullptr;
    tile_table(&tab);
    const TileEntry& T = tab[P->tile_index];
    hipError_t e = hipSuccess;
    for (int st = 0; st < 4; ++st) {
        if (P->any_ghost_fill && (e = launch_ghosts(P->ghosts[st], s)) != hipSuccess) return e;
        if ((e = T.launch(P->fused[st], P->prm, MODE_STAGE, st + 1, P->persistent, s)) != hipSuccess) return e;
        if (P->any_sommerfeld && (e = launch_sommerfeld(P->fused[st], P->prm, MODE_STAGE, st + 1, s)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// Validation of a box list shared by z4c_plan_create and z4c_autotune.
static int check_boxes(const z4c_box* boxes, int nbox)
{
    int rc;
    if (!boxes || nbox < 1 || nbox > MAXBOX) return fail(Z4C_EINVAL, "need 1..16 boxes");
    for (int b = 0; b < nbox; ++b) {
        const z4c_box& x = boxes[b];
        long stored = 0;
        const std::string tag = "box " + std::to_string(b) + ": ";
        if ((rc = check_geom(x.sf, x.n[0], x.n[1], x.n[2], x.ng, x.bc, &stored)) ||
            (rc = check_spacing(x.dx[0], x.dx[1], x.dx[2], x.x0[0], x.x0[1], x.x0[2])))
            return fail(rc, tag + g_last_error);
        if (!finite_pos(x.dt)) return fail(Z4C_EINVAL, tag + "dt must be finite and > 0");
        if (!x.u_n || !x.u_a || !x.u_b || !x.acc) return fail(Z4C_EINVAL, tag + "state buffers must be non-NULL");
        const void* bufs[4] = {x.u_n, x.u_a, x.u_b, x.acc};
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j)
                if (overlap(bufs[i], bufs[j], x.sf)) return fail(Z4C_EINVAL, tag + "state buffers overlap");
        if (x.bc == Z4C_BC_COPY && !x.shell) return fail(Z4C_EINVAL, tag + "copy box needs a shell");
        if (x.bc != Z4C_BC_COPY && x.shell) return fail(Z4C_EINVAL, tag + "shell must be NULL");
    }
    return Z4C_OK;
}

int z4c_plan_create(const z4c_box* boxes, int nbox, const z4c_params* p, const z4c_tile* tile,
                    const char* tune_cache_path, void** plan)
{
    int rc;
    if (!plan) return fail(Z4C_EINVAL, "plan is NULL");
    *plan = nullptr;
    if ((rc = check_params(p))) return rc;
    if ((rc = check_boxes(boxes, nbox))) return rc;
    z4c_tile chosen{};
    int source = Z4C_TILE_DEFAULT;
    if (tile) {
        chosen = *tile;
        source = Z4C_TILE_CALLER;
    } else if (tune_cache_path) {
        std::vector<TuneEntry> entries;
        if ((rc = tune_read(tune_cache_path, entries))) return rc;
        if (!entries.empty()) {  // a hit needs the device's architecture (the only HIP query here)
            std::string arch;
            if ((rc = device_arch(arch))) return rc;
            const TuneEntry* hit = tune_find(entries, arch, p->precision, nbox, cells_bucket(boxes, nbox));
            if (hit && find_tile(p->precision, &hit->tile) >= 0) {
                chosen = hit->tile;
                source = Z4C_TILE_CACHE;
            }
        }
    }
    int ti = source != Z4C_TILE_DEFAULT ? find_tile(p->precision, &chosen) : default_tile_index(p->precision);
    if (ti < 0) return fail(Z4C_EUNSUPPORTED, "no compiled tile of that shape for this precision");
    z4c_plan_s* P = new (std::nothrow) z4c_plan_s();
    if (!P) return fail(Z4C_ENOMEM, "plan allocation failed");
    P->boxes.assign(boxes, boxes + nbox);
    P->prm = to_dev(p);
    P->precision = p->precision;
    P->tile_index = ti;
    P->persistent = source != Z4C_TILE_DEFAULT ? (chosen.persistent ? 1 : 0) : 1;
    P->tile_source = source;
    P->any_ghost_fill = P->any_sommerfeld = false;
    for (const z4c_box& x : P->boxes) {
        P->any_ghost_fill |= x.bc != Z4C_BC_SOMMERFELD;
        P->any_sommerfeld |= x.bc == Z4C_BC_SOMMERFELD || x.bc == Z4C_BC_EQUATORIAL;
    }
    P->graph = nullptr;
    P->exec = nullptr;
    P->capture = nullptr;
    plan_build_sets(P);
    *plan = P;
    return Z4C_OK;
}

int z4c_plan_step(void* plan, int nsteps, int use_graph, void* stream)
{
    if (!plan) return fail(Z4C_EINVAL, "plan is NULL");
    if (nsteps < 0) return fail(Z4C_EINVAL, "nsteps must be >= 0");
    z4c_plan_s* P = (z4c_plan_s*)plan;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pending HIP error before z4c_plan_step");
    if (!use_graph) {
        for (int i = 0; i < nsteps; ++i)
            if ((e = plan_enqueue_step(P, s)) != hipSuccess) return hip_fail(e, "plan step launch");
        return Z4C_OK;
    }
    if (nsteps == 0) return Z4C_OK;
    if (!P->exec) {
        // Capture one RK4 step on a private stream (the legacy default stream
        // cannot be captured); the instantiated graph is launched on `s`.
        if (!P->capture && (e = hipStreamCreateWithFlags(&P->capture, hipStreamNonBlocking)) != hipSuccess) {
            P->capture = nullptr;
            return hip_fail(e, "hipStreamCreateWithFlags");
        }
        if ((e = hipStreamBeginCapture(P->capture, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "hipStreamBeginCapture");
        hipError_t le = plan_enqueue_step(P, P->capture);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(P->capture, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(le, "plan step launch during capture");
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        hipGraphExec_t x = nullptr;
        if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        P->graph = g;
        P->exec = x;
    }
    for (int i = 0; i < nsteps; ++i)
        if ((e = hipGraphLaunch(P->exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return Z4C_OK;
}

static int plan_autotune_impl(void* plan, int reps, void* stream, z4c_tile* best, float* ms, float* best_ms_out)
{
    if (!plan) return fail(Z4C_EINVAL, "plan is NULL");
    if (reps < 1 || reps > 1000) return fail(Z4C_EINVAL, "reps must be 1..1000");
    z4c_plan_s* P = (z4c_plan_s*)plan;
    hipStream_t s = (hipStream_t)stream;
    const TileEntry* tab = nullptr;
    const int n = tile_table(&tab);
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return hip_fail(e, "hipEventCreate");
    }
    const int keep = P->tile_index, keep_p = P->persistent;
    int best_i = -1, best_p = 0;
    float best_ms = 0.0f;
    int c = 0;
    for (int i = 0; i < n; ++i) {
        if (tab[i].precision != P->precision) continue;
        for (int pers = 0; pers < 2; ++pers, ++c) {
            P->tile_index = i;
            P->persistent = pers;
            plan_drop_graph(P);
            plan_build_sets(P);
            std::vector<float> t;
            e = plan_enqueue_step(P, s);  // warm-up
            for (int r = 0; r < reps && e == hipSuccess; ++r) {
                (void)hipEventRecord(a, s);
                e = plan_enqueue_step(P, s);
                (void)hipEventRecord(b, s);
                if (e == hipSuccess) e = hipEventSynchronize(b);
                float x = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&x, a, b);
                t.push_back(x);
            }
            if (e != hipSuccess) {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
                P->tile_index = keep;
                P->persistent = keep_p;
                plan_build_sets(P);
                return hip_fail(e, "autotune trial");
            }
            std::sort(t.begin(), t.end());
            const float med = t[t.size() / 2];
            if (ms) ms[c] = med;
            if (best_i < 0 || med < best_ms) {
                best_i = i;
                best_p = pers;
                best_ms = med;
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    P->tile_index = best_i;
    P->persistent = best_p;
    P->tile_source = Z4C_TILE_TUNED;
    plan_drop_graph(P);
    plan_build_sets(P);
    if (best_ms_out) *best_ms_out = best_ms;
    if (best) {
        *best = tab[best_i].tile;
        best->persistent = best_p;
    }
    return Z4C_OK;
}

int z4c_plan_autotune(void* plan, int reps, void* stream, z4c_tile* best, float* ms)
{
    return plan_autotune_impl(plan, reps, stream, best, ms, nullptr);
}

int z4c_plan_tile(void* plan, z4c_tile* tile, int* source)
{
    if (!plan) return fail(Z4C_EINVAL, "plan is NULL");
    const z4c_plan_s* P = (const z4c_plan_s*)plan;
    const TileEntry* tab = nullptr;
    tile_table(&tab);
    if (tile) {
        *tile = tab[P->tile_index].tile;
        tile->persistent = P->persistent;
    }
    if (source) *source = P->tile_source;
    return Z4C_OK;
}

int z4c_tune_lookup(const char* tune_cache_path, const char* arch, const z4c_box* boxes, int nbox, int precision,
                    z4c_tile* tile)
{
    int rc;
    if (!tune_cache_path || !arch || !tile) return fail(Z4C_EINVAL, "tune_cache_path, arch and tile must be non-NULL");
    if (precision != Z4C_FP64 && precision != Z4C_MIXED) return fail(Z4C_EINVAL, "unknown precision");
    if (!boxes || nbox < 1 || nbox > MAXBOX) return fail(Z4C_EINVAL, "need 1..16 boxes");
    for (int b = 0; b < nbox; ++b)
        if (boxes[b].n[0] < 1 || boxes[b].n[1] < 1 || boxes[b].n[2] < 1)
            return fail(Z4C_EINVAL, "active extents must be >= 1");
    std::vector<TuneEntry> v;
    if ((rc = tune_read(tune_cache_path, v))) return rc;
    const TuneEntry* e = tune_find(v, arch, precision, nbox, cells_bucket(boxes, nbox));
    if (!e || find_tile(precision, &e->tile) < 0) return 0;
    *tile = e->tile;
    return 1;
}

int z4c_autotune(const z4c_box* boxes, int nbox, const z4c_params* p, const char* tune_cache_path, void* stream,
                 z4c_tile* best, int* source)
{
    int rc;
    if ((rc = check_params(p))) return rc;
    if ((rc = check_boxes(boxes, nbox))) return rc;
    std::vector<TuneEntry> entries;
    if (tune_cache_path && (rc = tune_read(tune_cache_path, entries))) return rc;
    std::string arch;
    if ((rc = device_arch(arch))) return rc;
    const int bucket = cells_bucket(boxes, nbox);
    const TuneEntry* hit = tune_find(entries, arch, p->precision, nbox, bucket);
    if (hit && find_tile(p->precision, &hit->tile) >= 0) {
        if (best) *best = hit->tile;
        if (source) *source = Z4C_TILE_CACHE;
        return Z4C_OK;
    }
    void* plan = nullptr;
    if ((rc = z4c_plan_create(boxes, nbox, p, nullptr, nullptr, &plan))) return rc;
    z4c_tile t{};
    float ms = 0.0f;
    rc = plan_autotune_impl(plan, 2, stream, &t, nullptr, &ms);
    const std::string err = g_last_error;
    z4c_plan_destroy(plan);
    if (rc) return fail(rc, err);
    if (tune_cache_path) {
        TuneEntry e;
        e.arch = arch;
        e.precision = p->precision;
        e.nbox = nbox;
        e.bucket = bucket;
        e.tile = t;
        e.ms = ms;
        if ((rc = tune_write(tune_cache_path, e))) return rc;
    }
    if (best) *best = t;
    if (source) *source = Z4C_TILE_TUNED;
    return Z4C_OK;
}

int z4c_plan_destroy(void* plan)
{
    if (!plan) return fail(Z4C_EINVAL, "plan is NULL");
    z4c_plan_s* P = (z4c_plan_s*)plan;
    plan_drop_graph(P);
    if (P->capture) (void)hipStreamDestroy(P->capture);
    delete P;
    return Z4C_OK;
}

// ---------------------------------------------------------------------------
// Box-in-box hierarchy with Berger-Oliger subcycling
// ---------------------------------------------------------------------------
namespace {
constexpr int MAXPATCH = 32;
}

struct HierPatch {
    z4c_level L;
    double* lev[3];  // device: spatial prolongations of the parent's time levels (prev, cur, new)
    double wt[3];    // their weights at the current stage time (wt[0] unused without prev)
    bool quad;       // the parent holds prev: quadratic in time
    bool lev_cur;    // lev[1] holds the prolongation of the parent's cur of its previous step, at this geometry
    long nshell;
    bool has_prev;  // prev holds this patch one step earlier
    bool plane;     // its lower z face is the symmetry plane of an equatorial root
    int depth;
    int off[3];     // lattice index of the first active cell at the patch's depth
};

struct HierDepth {
    std::vector<int> q;  // its patches, in index order
    BoxSet fused[4];
    BoxSet fill[4];      // ghost fill of the stage inputs u, a, b, a
    BoxSet mirror[4];    // the patches on the symmetry plane: their layers below it
};

struct z4c_hier_s {
    std::vector<HierPatch> pt;
    std::vector<HierDepth> dp;
    ParamsDev prm;
    int precision;
    int tile_index;
    int persistent;
    double dt0;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t capture;
    int nobj;            // tracked objects (0: no moving patches)
    int tp[MAXEX];       // per object: the patch it is tracked on
    double* track;       // device: per object x[3], b0[3], xs[3], error flag
    double* sepx;        // device scratch of the separable prolongation (x sums)
    double* sepy;        // (y sums)
    size_t sepx_cap, sepy_cap;  // their lengths (doubles)
};

// Parent rows (active index, before reflection) read by the prolongation of
// child cells a = a0 .. a1 - 1 along one direction with faces on parent cell F.
static void prolong_rows(int F, int a0, int a1, int& lo, int& hi)
{
    lo = INT32_MAX;
    hi = INT32_MIN;
    for (int a = a0; a < a1; ++a) {
        const int half = a >= 0 ? a / 2 : -((1 - a) / 2);
        const bool odd = a - 2 * half != 0;
        lo = std::min(lo, F + half + (odd ? -2 : -3));
        hi = std::max(hi, F + half + (odd ? 3 : 2));
    }
}

// Parent rows that the lower (child index -ng .. -1) and upper (n .. n+ng-1)
// ghost layers of a child read along one direction: {lo0, hi0, lo1, hi1};
// refl maps a row r < 0 to its mirror image -1 - r.
static void face_rows(int F, int n, int ng, bool refl, int out[4])
{
    auto span = [&](int a0, int a1, int& lo, int& hi) {
        lo = INT32_MAX;
        hi = INT32_MIN;
        for (int a = a0; a < a1; ++a) {
            const int half = a >= 0 ? a / 2 : -((1 - a) / 2);
            const bool odd = a - 2 * half != 0;
            for (int o = odd ? -2 : -3; o <= (odd ? 3 : 2); ++o) {
                int r = F + half + o;
                if (refl && r < 0) r = -1 - r;
                lo = std::min(lo, r);
                hi = std::max(hi, r);
            }
        }
    };
    span(-ng, 0, out[0], out[1]);
    span(n, n + ng, out[2], out[3]);
}

// the scratch window of patch P: parent y rows Y0 .. Y0+NY-1, z rows Z0 .. Z0+NZ-1
static void sep_window(const z4c_level& L, bool plane, int& Y0, int& NY, int& Z0, int& NZ)
{
    int lo, hi;
    prolong_rows(L.F[1], -L.ng, L.n[1] + L.ng, lo, hi);
    Y0 = lo;
    NY = hi - lo + 1;
    prolong_rows(L.F[2], -L.ng, L.n[2] + L.ng, lo, hi);
    if (plane && lo < 0) {  // rows below the symmetry plane are read reflected
        hi = std::max(hi, -1 - lo);
        lo = 0;
    }
    Z0 = lo;
    NZ = hi - lo + 1;
}

// Geometry of patch x against its parent P: 2:1 spacing, lower faces on
// parent cell F, every ghost's prolongation stencil in P's active cells.
static int hier_check_level(const z4c_level& x, const z4c_level& P, bool plane, const std::string& tag)
{
    for (int d = 0; d < 3; ++d) {
        if (x.n[d] % 2) return fail(Z4C_EINVAL, tag + "active extents must be even");
        if (x.dx[d] != 0.5 * P.dx[d]) return fail(Z4C_EINVAL, tag + "dx must be half the parent's");
        const double want = P.x0[d] + (x.F[d] - 0.25) * P.dx[d];
        if (std::fabs(x.x0[d] - want) > 1e-9 * P.dx[d])
            return fail(Z4C_EINVAL, tag + "x0 does not put the lower faces on parent cell F");
        // first / last parent cell read by the ghost stencils: child cell a
        // lies in parent cell F + floor(a/2), in its upper half for odd a
        // (stencil -2..+3) and its lower half for even a (-3..+2)
        auto span = [](int a, int& from, int& to) {
            const int half = a >= 0 ? a / 2 : -((1 - a) / 2);
            const bool odd = a - 2 * half != 0;
            from = half + (odd ? -2 : -3);
            to = half + (odd ? 3 : 2);
        };
        int lo_from, lo_to, hi_from, hi_to;
        span(-x.ng, lo_from, lo_to);
        span(x.n[d] + x.ng - 1, hi_from, hi_to);
        int lo = x.F[d] + lo_from;
        const int hi = x.F[d] + hi_to;
        if (d == 2 && plane && lo < 0) lo = -1 - lo;  // layers below the symmetry plane read as mirror images
        if (lo < 0 || lo >= P.n[d] || hi >= P.n[d])
            return fail(Z4C_EINVAL, tag + "prolongation stencil leaves the parent's active cells");
    }
    return Z4C_OK;
}

// depths, lattice offsets and the per-depth patch lists
static void hier_geometry(z4c_hier_s* H)
{
    int maxd = 0;
    for (size_t q = 0; q < H->pt.size(); ++q) {
        HierPatch& P = H->pt[q];
        if (q == 0) {
            P.depth = 0;
            P.plane = P.L.bc == Z4C_BC_EQUATORIAL;
            for (int d = 0; d < 3; ++d) P.off[d] = 0;
            continue;
        }
        const HierPatch& R = H->pt[P.L.parent];
        P.depth = R.depth + 1;
        P.plane = R.plane && P.L.F[2] == 0;
        maxd = std::max(maxd, P.depth);
        // child active cell a sits at lattice index 2 (parent's first cell + F) + a
        for (int d = 0; d < 3; ++d) P.off[d] = 2 * (R.off[d] + P.L.F[d]);
    }
    H->dp.resize(maxd + 1);
    for (HierDepth& D : H->dp) D.q.clear();
    for (size_t q = 0; q < H->pt.size(); ++q) H->dp[H->pt[q].depth].q.push_back((int)q);
}

// stage inputs and outputs of the four stages: u -> a -> b -> a -> u
static double* stage_in(const z4c_level& L, int st)
{
    return st == 0 ? L.u : (st == 2 ? L.u_b : L.u_a);
}
static double* stage_out(const z4c_level& L, int st)
{
    return st == 0 ? L.u_a : (st == 1 ? L.u_b : (st == 2 ? L.u_a : L.u));
}

// (Re)build the stage and ghost-fill sets of depth d from its patches.
static void hier_build_sets(z4c_hier_s* H, int d)
{
    const TileEntry* tab = nullptr;
    tile_table(&tab);
    HierDepth& D = H->dp[d];
    const double dt = H->dt0 / (double)(1L << d);
    for (int st = 0; st < 4; ++st) {
        BoxSet& F = D.fused[st];
        F = BoxSet{};
        F.nbox = (int)D.q.size();
        for (int b = 0; b < F.nbox; ++b) {
            const HierPatch& P = H->pt[D.q[b]];
            BoxDev x = make_box(P.L.n, P.L.ng, P.L.bc, P.L.sf, P.L.dx, P.L.x0, dt);
            x.u_in = stage_in(P.L, st);
            x.u_n = P.L.u;
            x.acc = P.L.acc;
            x.u_out = stage_out(P.L, st);
            F.box[b] = x;
        }
        finalize_set(F, tab[H->tile_index].tile);
        D.fill[st] = F;
        BoxSet& M = D.mirror[st];
        M = BoxSet{};
        for (int b = 0; b < F.nbox; ++b)
            if (D.q[b] > 0 && H->pt[D.q[b]].plane) {
                M.box[M.nbox] = F.box[b];
                M.box[M.nbox].bc = Z4C_BC_EQUATORIAL;
                ++M.nbox;
            }
        finalize_set(M, tab[H->tile_index].tile);
    }
}

static PatchRef patch_ref(const HierPatch& P, double* arr)
{
    PatchRef r{};
    r.u = arr;
    r.sf = P.L.sf;
    r.ng = P.L.ng;
    for (int d = 0; d < 3; ++d) {
        r.N[d] = P.L.n[d] + 2 * P.L.ng;
        r.n[d] = P.L.n[d];
        r.off[d] = P.off[d];
    }
    return r;
}

// intersection of the lattice box [lo, lo + ext) with the bounding box of
// the active regions of the depth's patches other than t; false if empty
static bool others_box(const ExchArgs& a, int lo[3], int ext[3])
{
    int blo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, bhi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (int b = 0; b < a.np; ++b) {
        if (b == a.t) continue;
        for (int d = 0; d < 3; ++d) {
            blo[d] = std::min(blo[d], a.p[b].off[d]);
            bhi[d] = std::max(bhi[d], a.p[b].off[d] + a.p[b].n[d]);
        }
    }
    for (int d = 0; d < 3; ++d) {
        const int l = std::max(lo[d], blo[d]), h = std::min(lo[d] + ext[d], bhi[d]);
        if (h <= l) return false;
        lo[d] = l;
        ext[d] = h - l;
    }
    return true;
}

// exchange at depth d on the stage-st input arrays: ghosts inside another
// patch's active region take its values
static hipError_t hier_exchange_ghosts(z4c_hier_s* H, int d, int st, hipStream_t s)
{
    const HierDepth& D = H->dp[d];
    if (D.q.size() < 2) return hipSuccess;
    ExchArgs a{};
    a.np = (int)D.q.size();
    for (int b = 0; b < a.np; ++b) a.p[b] = patch_ref(H->pt[D.q[b]], stage_in(H->pt[D.q[b]].L, st));
    for (int t = 0; t < a.np; ++t) {
        a.t = t;
        for (int e = 0; e < 3; ++e) {
            a.lo[e] = a.p[t].off[e] - a.p[t].ng;
            a.ext[e] = a.p[t].N[e];
        }
        if (!others_box(a, a.lo, a.ext)) continue;
        hipError_t e = launch_exchange_ghosts(a, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// exchange at depth d on the states: overlapping active cells take their mean
static hipError_t hier_exchange_average(z4c_hier_s* H, int d, hipStream_t s)
{
    const HierDepth& D = H->dp[d];
    if (D.q.size() < 2) return hipSuccess;
    ExchArgs a{};
    a.np = (int)D.q.size();
    for (int b = 0; b < a.np; ++b) a.p[b] = patch_ref(H->pt[D.q[b]], H->pt[D.q[b]].L.u);
    for (int t = 0; t < a.np; ++t) {
        a.t = t;
        for (int e = 0; e < 3; ++e) {
            a.lo[e] = a.p[t].off[e];
            a.ext[e] = a.p[t].n[e];
        }
        if (!others_box(a, a.lo, a.ext)) continue;
        hipError_t e = launch_exchange_average(a, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// the puncture update (mode 0: predictor, 1: corrector) of every object
// whose deepest patch is at depth d, in one launch
static hipError_t hier_track(z4c_hier_s* H, int d, int mode, hipStream_t s)
{
    TrackBatch b{};
    for (int o = 0; o < H->nobj; ++o) {
        const HierPatch& P = H->pt[H->tp[o]];
        if (P.depth != d) continue;
        TrackArgs& a = b.a[b.n++];
        a.state = H->track + 10 * o;
        a.u = P.L.u;
        a.sf = P.L.sf;
        for (int e = 0; e < 3; ++e) {
            a.N[e] = P.L.n[e] + 2 * P.L.ng;
            a.x0[e] = P.L.x0[e];
            a.h[e] = P.L.dx[e];
        }
        a.ng = P.L.ng;
        a.dt = H->dt0 / (double)(1L << P.depth);
        a.mode = mode;
        a.refl = P.plane ? 1 : 0;
    }
    return launch_track(b, s);
}

// Lagrange weights of the parent time levels (nodes -1, 0, 1 in units of
// the parent step) at theta; linear in (0, 1) without an earlier level.
static void hier_time_weights(double theta, bool quadratic, double wt[3])
{
    if (quadratic) {
        wt[0] = 0.5 * theta * (theta - 1.0);
        wt[1] = (1.0 - theta) * (1.0 + theta);
        wt[2] = 0.5 * theta * (theta + 1.0);
    } else {
        wt[0] = 0.0;
        wt[1] = 1.0 - theta;
        wt[2] = theta;
    }
}

// The ghost shells of every patch at depth d at theta (fraction of the
// parent step).  Prolongation in space and interpolation in time are both
// linear and commute: at the start of a parent step (theta 0) each parent
// time level is prolonged once into its own shell; the shell of every stage
// time is their weighted sum, formed by the ghost fill with the weights set
// here.
static hipError_t hier_prolong(z4c_hier_s* H, int d, double theta, hipStream_t s)
{
    hipError_t e;
    if (theta == 0.0) {
        // the parent's prev is its cur of the previous step: reuse that
        // prolongation unless the patch moved since (copied before lev[1]
        // is overwritten below)
        CopyList reuse{};
        for (int q : H->dp[d].q) {
            const HierPatch& C = H->pt[q];
            if (!(H->pt[C.L.parent].has_prev && C.lev_cur)) continue;
            reuse.dst[reuse.n] = C.lev[0];
            reuse.src[reuse.n] = C.lev[1];
            reuse.len[reuse.n] = (long)NF * C.nshell;
            reuse.begin[reuse.n + 1] = batch_add(reuse.begin[reuse.n], reuse.len[reuse.n]);
            ++reuse.n;
        }
        if ((e = launch_copy_list(reuse, s)) != hipSuccess) return e;
        // every other level of every patch: the separable passes in batches
        // that share the scratch (a batch's passes are done before the next
        // batch's first pass, on the same stream)
        SepBatch b{};
        size_t ox = 0, oy = 0;
        for (int q : H->dp[d].q) {
            HierPatch& C = H->pt[q];
            const HierPatch& P = H->pt[C.L.parent];
            const double* lv[3] = {P.L.prev, P.L.cur, P.L.u};
            const bool reused = P.has_prev && C.lev_cur;
            for (int t = P.has_prev && !reused ? 0 : 1; t < 3; ++t) {
                SepArgs a{};
                a.u = lv[t];
                a.sfp = P.L.sf;
                for (int k = 0; k < 3; ++k) {
                    a.Np[k] = P.L.n[k] + 2 * P.L.ng;
                    a.nc[k] = C.L.n[k];
                    a.F[k] = C.L.F[k];
                }
                a.ngp = P.L.ng;
                a.ngc = C.L.ng;
                sep_window(C.L, C.plane, a.Y0, a.NY, a.Z0, a.NZ);
                a.shell = C.lev[t];
                a.nshell = C.nshell;
                a.refl = C.plane ? 1 : 0;
                face_rows(C.L.F[2], C.L.n[2], C.L.ng, C.plane, a.zf);
                face_rows(C.L.F[1], C.L.n[1], C.L.ng, false, a.yf);
                long nx, ny, nz;
                sep_counts(a, nx, ny, nz);
                const size_t sx = (size_t)NF * nx, sy = (size_t)NF * ny;  // scratch of all fields
                if (b.n == MAXSEP || ox + sx > H->sepx_cap || oy + sy > H->sepy_cap) {
                    if ((e = launch_prolong_sep(b, s)) != hipSuccess) return e;
                    b = SepBatch{};
                    ox = oy = 0;
                }
                a.X = H->sepx + ox;
                a.Y = H->sepy + oy;
                ox += sx;
                oy += sy;
                b.e[b.n] = a;
                b.bx[b.n + 1] = batch_add(b.bx[b.n], nx);
                b.by[b.n + 1] = batch_add(b.by[b.n], ny);
                b.bz[b.n + 1] = batch_add(b.bz[b.n], nz);
                ++b.n;
            }
            C.lev_cur = true;
        }
        if ((e = launch_prolong_sep(b, s)) != hipSuccess) return e;
    }
    for (int q : H->dp[d].q) {
        HierPatch& C = H->pt[q];
        C.quad = H->pt[C.L.parent].has_prev;
        hier_time_weights(theta, C.quad, C.wt);
    }
    return hipSuccess;
}

// the ghost fill of stage input st at depth d: copy boxes take the weighted
// sum of their parent's time levels at the stage time of their last
// hier_prolong (the weights are kernel arguments, so a captured graph keeps
// each launch's own)
static BoxSet hier_fill_set(const z4c_hier_s* H, int d, int st)
{
    BoxSet F = H->dp[d].fill[st];
    for (int b = 0; b < F.nbox; ++b) {
        const HierPatch& C = H->pt[H->dp[d].q[b]];
        if (H->dp[d].q[b] == 0) continue;
        // theta 0 and 1 fall on the parent's cur and new levels: a copy
        const int only = C.wt[0] == 0.0 && C.wt[1] == 1.0 && C.wt[2] == 0.0   ? 1
                         : C.wt[0] == 0.0 && C.wt[1] == 0.0 && C.wt[2] == 1.0 ? 2
                                                                              : -1;
        if (only > 0) {
            F.box[b].lv[1] = C.lev[only];
            continue;
        }
        F.box[b].lv[0] = C.quad ? C.lev[0] : nullptr;
        F.box[b].lv[1] = C.lev[1];
        F.box[b].lv[2] = C.lev[2];
        for (int t = 0; t < 3; ++t) F.box[b].lw[t] = C.wt[t];
    }
    return F;
}

// The parent cells (stored coordinates of P) that the prolongation of its
// child C reads, one cell wider where C may shift (by one parent cell at
// most, at a root-step boundary) before a level kept now is read again.
static void child_window(const HierPatch& P, const HierPatch& C, int lo[3], int ext[3])
{
    for (int d = 0; d < 3; ++d) {
        int l, h;
        prolong_rows(C.L.F[d], -C.L.ng, C.L.n[d] + C.L.ng, l, h);
        if (d == 2 && C.plane && l < 0) {  // rows below the symmetry plane are read reflected
            h = std::max(h, -1 - l);
            l = 0;
        }
        if (C.L.obj >= 0 && !(d == 2 && C.plane)) {
            --l;
            ++h;
        }
        l = std::max(l + P.L.ng, 0);
        h = std::min(h + P.L.ng, P.L.n[d] + 2 * P.L.ng - 1);
        lo[d] = l;
        ext[d] = h - l + 1;
    }
}

// keep a time level of every patch at depth d (prev: prev <- cur, else
// cur <- u), over the cells their children's prolongations read, in one launch
static hipError_t hier_keep_levels(z4c_hier_s* H, int d, bool prev, hipStream_t s)
{
    CopyBoxBatch b{};
    for (int c : H->dp[d + 1].q) {
        const HierPatch& C = H->pt[c];
        const HierPatch& P = H->pt[C.L.parent];
        CopyBoxArgs& a = b.e[b.n];
        a.dst = prev ? P.L.prev : P.L.cur;
        a.src = prev ? P.L.cur : P.L.u;
        a.sf = P.L.sf;
        for (int e = 0; e < 3; ++e) a.N[e] = P.L.n[e] + 2 * P.L.ng;
        child_window(P, C, a.lo, a.ext);
        b.begin[b.n + 1] = batch_add(b.begin[b.n], (long)NF * a.ext[0] * a.ext[1] * a.ext[2]);
        ++b.n;
    }
    return launch_copy_box(b, s);
}

// every patch at depth d: the cells covered by the patches of depth d+1
static hipError_t hier_restrict(z4c_hier_s* H, int d, hipStream_t s)
{
    const HierDepth& C = H->dp[d + 1];
    RestrictArgs a{};
    a.nchild = (int)C.q.size();
    int clo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, chi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (int c = 0; c < a.nchild; ++c) {
        a.child[c] = patch_ref(H->pt[C.q[c]], H->pt[C.q[c]].L.u);
        for (int e = 0; e < 3; ++e) {  // covered lattice cells of depth d (off and n are even)
            clo[e] = std::min(clo[e], a.child[c].off[e] / 2);
            chi[e] = std::max(chi[e], (a.child[c].off[e] + a.child[c].n[e]) / 2);
        }
    }
    for (int q : H->dp[d].q) {
        const HierPatch& P = H->pt[q];
        a.parent = patch_ref(P, P.L.u);
        bool empty = false;
        for (int e = 0; e < 3; ++e) {
            const int l = std::max(0, clo[e] - P.off[e]), h = std::min(P.L.n[e], chi[e] - P.off[e]);
            empty |= h <= l;
            a.lo[e] = l;
            a.ext[e] = h - l;
        }
        if (empty) continue;
        hipError_t e = launch_restrict(a, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// One RK4 step of every patch at depth d starting at theta0 (fraction of
// the parent step), then, if there is a finer depth, its two steps, its
// ghost fill at the end time and the restriction.  Stage inputs get their
// ghosts (prolongation, then the exchange) at the stage times theta0 + {0,
// 1/4, 1/4, 1/2}; overlapping active cells are averaged after the last stage.
static hipError_t hier_depth_step(z4c_hier_s* H, int d, double theta0, hipStream_t s)
{
    const TileEntry* tab = nullptr;
    tile_table(&tab);
    const TileEntry& T = tab[H->tile_index];
    HierDepth& D = H->dp[d];
    const int ndepth = (int)H->dp.size();
    const z4c_level& R = H->pt[0].L;
    const bool outer = d == 0 && (R.bc == Z4C_BC_SOMMERFELD || R.bc == Z4C_BC_EQUATORIAL);
    hipError_t e;
    // Patches (copy boxes) fill two arrays at once where two consumers share
    // a stage time:
    // * stage inputs 1 and 2, before stage 1 (which writes only the active
    //   cells of input 2);
    // * stage input 3 and the state u, whose next ghosts are taken at the same
    //   time: at the start of the second step of the pair (theta 1/2), or by
    //   the parent after the pair (theta 1).  Until then only active cells of
    //   u are written or read (last stage, mean of overlaps, tracking, the
    //   children's windows, restriction).
    // The exchange and the mirror of the second array still follow the
    // stages before its use, since they read active cells.
    auto fill = [&](int st) -> hipError_t {
        hipError_t r = hipSuccess;
        if (d > 0 && (st == 1 || st == 3)) {
            BoxSet F = hier_fill_set(H, d, st);
            for (int b = 0; b < F.nbox; ++b) F.box[b].u_in2 = stage_in(H->pt[D.q[b]].L, st == 1 ? 2 : 0);
            r = launch_ghosts(F, s);
        } else {
            const bool root_evolved = d == 0 && R.bc == Z4C_BC_SOMMERFELD;  // outer ghosts are evolved
            const bool filled_before = d > 0 && (st == 2 || (st == 0 && theta0 != 0.0));
            if (!root_evolved && !filled_before) r = launch_ghosts(hier_fill_set(H, d, st), s);
        }
        if (r == hipSuccess) r = hier_exchange_ghosts(H, d, st, s);
        if (r == hipSuccess && D.mirror[st].nbox) r = launch_ghosts(D.mirror[st], s);
        return r;
    };
    auto stage = [&](int st) -> hipError_t {
        hipError_t r = T.launch(D.fused[st], H->prm, MODE_STAGE, st + 1, H->persistent, s);
        if (r == hipSuccess && outer) r = launch_sommerfeld(D.fused[st], H->prm, MODE_STAGE, st + 1, s);
        return r;
    };
    if (d > 0 && theta0 == 0.0 && (e = hier_prolong(H, d, 0.0, s)) != hipSuccess) return e;
    if ((e = fill(0)) != hipSuccess) return e;
    if (d + 1 < ndepth && (e = hier_keep_levels(H, d, false, s)) != hipSuccess) return e;
    if ((e = hier_track(H, d, 0, s)) != hipSuccess) return e;
    if ((e = stage(0)) != hipSuccess) return e;
    if (d > 0 && (e = hier_prolong(H, d, theta0 + 0.25, s)) != hipSuccess) return e;
    if ((e = fill(1)) != hipSuccess || (e = stage(1)) != hipSuccess) return e;
    if ((e = fill(2)) != hipSuccess || (e = stage(2)) != hipSuccess) return e;
    if (d > 0 && (e = hier_prolong(H, d, theta0 + 0.5, s)) != hipSuccess) return e;
    if ((e = fill(3)) != hipSuccess || (e = stage(3)) != hipSuccess) return e;
    if ((e = hier_exchange_average(H, d, s)) != hipSuccess) return e;
    if ((e = hier_track(H, d, 1, s)) != hipSuccess) return e;
    if (d + 1 < ndepth) {
        if ((e = hier_depth_step(H, d + 1, 0.0, s)) != hipSuccess) return e;
        if ((e = hier_depth_step(H, d + 1, 0.5, s)) != hipSuccess) return e;
        // the patches' ghosts at theta 1 were filled with their last stage input
        if ((e = hier_exchange_ghosts(H, d + 1, 0, s)) != hipSuccess) return e;
        if (H->dp[d + 1].mirror[0].nbox && (e = launch_ghosts(H->dp[d + 1].mirror[0], s)) != hipSuccess) return e;
        if ((e = hier_restrict(H, d, s)) != hipSuccess) return e;
        if ((e = hier_keep_levels(H, d, true, s)) != hipSuccess) return e;
        for (int q : D.q) H->pt[q].has_prev = true;
    }
    return hipSuccess;
}

static void hier_drop_graph(z4c_hier_s* H)
{
    if (H->exec) (void)hipGraphExecDestroy(H->exec);
    if (H->graph) (void)hipGraphDestroy(H->graph);
    H->exec = nullptr;
    H->graph = nullptr;
}

static void hier_free(z4c_hier_s* H)
{
    hier_drop_graph(H);
    for (HierPatch& P : H->pt) {
        for (double* b : P.lev)
            if (b) (void)hipFree(b);
    }
    if (H->track) (void)hipFree(H->track);
    if (H->sepx) (void)hipFree(H->sepx);
    if (H->sepy) (void)hipFree(H->sepy);
    if (H->capture) (void)hipStreamDestroy(H->capture);
    delete H;
}

int z4c_hier_create(const z4c_level* levels, int nlev, const z4c_params* p, double dt0, const z4c_tile* tile,
                    void** hier)
{
    int rc;
    if (!hier) return fail(Z4C_EINVAL, "hier is NULL");
    *hier = nullptr;
    if ((rc = check_params(p))) return rc;
    if (!levels || nlev < 1 || nlev > MAXPATCH) return fail(Z4C_EINVAL, "need 1..32 patches");
    if (!finite_pos(dt0)) return fail(Z4C_EINVAL, "dt0 must be finite and > 0");
    std::vector<int> depth(nlev, 0);
    std::vector<char> plane(nlev, 0);
    for (int l = 0; l < nlev; ++l) {
        const z4c_level& x = levels[l];
        const std::string tag = "patch " + std::to_string(l) + ": ";
        long stored = 0;
        if ((rc = check_geom(x.sf, x.n[0], x.n[1], x.n[2], x.ng, x.bc, &stored)) ||
            (rc = check_spacing(x.dx[0], x.dx[1], x.dx[2], x.x0[0], x.x0[1], x.x0[2])))
            return fail(rc, tag + z4c_last_error());
        const double* arr[6] = {x.u, x.u_a, x.u_b, x.acc, x.prev, x.cur};
        for (int i = 0; i < 6; ++i) {
            if (!arr[i]) return fail(Z4C_EINVAL, tag + "all six state arrays are required");
            for (int j = 0; j < i; ++j)
                if (overlap(arr[i], arr[j], x.sf)) return fail(Z4C_EINVAL, tag + "state arrays overlap");
            for (int m = 0; m < l; ++m) {
                const z4c_level& y = levels[m];
                const double* brr[6] = {y.u, y.u_a, y.u_b, y.acc, y.prev, y.cur};
                for (int j = 0; j < 6; ++j)
                    if (overlap2(arr[i], x.sf, brr[j], y.sf))
                        return fail(Z4C_EINVAL, tag + "state arrays overlap those of patch " + std::to_string(m));
            }
        }
        if (x.obj < -1) return fail(Z4C_EINVAL, tag + "obj must be -1 (fixed) or a tracked object index");
        if (l == 0) {
            if (x.parent != -1) return fail(Z4C_EINVAL, tag + "the root (patch 0) has parent -1");
            if (x.bc == Z4C_BC_COPY) return fail(Z4C_EINVAL, tag + "the root needs its own boundary");
            if (x.obj != -1) return fail(Z4C_EINVAL, tag + "the root cannot move");
            plane[0] = x.bc == Z4C_BC_EQUATORIAL;
            continue;
        }
        if (x.parent < 0 || x.parent >= l) return fail(Z4C_EINVAL, tag + "parent must be a patch listed before it");
        if (x.bc != Z4C_BC_COPY) return fail(Z4C_EINVAL, tag + "patches >= 1 take Z4C_BC_COPY (filled from the parent)");
        plane[l] = plane[x.parent] && x.F[2] == 0;
        if ((rc = hier_check_level(x, levels[x.parent], plane[l], tag))) return rc;
        depth[l] = depth[x.parent] + 1;
        if (depth[l] > 30) return fail(Z4C_EINVAL, tag + "deeper than 30 levels");
    }
    for (int dd = 0; dd <= 30; ++dd)
        if (std::count(depth.begin(), depth.end(), dd) > MAXEX)
            return fail(Z4C_EINVAL, "more than 16 patches at depth " + std::to_string(dd));
    int pers = 1;
    int ti;
    if (tile) {
        ti = find_tile(p->precision, tile);
        if (ti < 0) return fail(Z4C_EUNSUPPORTED, "tile shape not compiled for this precision");
        pers = tile->persistent ? 1 : 0;
    } else {
        ti = default_tile_index(p->precision);
        if (ti < 0) return fail(Z4C_EUNSUPPORTED, "no tile compiled for this precision");
    }
    z4c_hier_s* H = new z4c_hier_s{};
    H->prm = to_dev(p);
    H->precision = p->precision;
    H->tile_index = ti;
    H->persistent = pers;
    H->dt0 = dt0;
    H->pt.resize(nlev);
    for (int l = 0; l < nlev; ++l) {
        HierPatch& P = H->pt[l];
        P.L = levels[l];
        P.lev[0] = P.lev[1] = P.lev[2] = nullptr;
        P.wt[0] = P.wt[1] = P.wt[2] = 0.0;
        P.quad = false;
        P.lev_cur = false;
        P.has_prev = false;
        P.nshell = l > 0 ? shell_size(P.L.n, P.L.ng) : 0;
    }
    for (int l = 1; l < nlev; ++l) {
        HierPatch& P = H->pt[l];
        double** bufs[3] = {&P.lev[0], &P.lev[1], &P.lev[2]};
        for (double** b : bufs) {
            const hipError_t e = hipMalloc((void**)b, (size_t)NF * P.nshell * sizeof(double));
            if (e != hipSuccess) {
                *b = nullptr;
                hier_free(H);
                return fail(Z4C_ENOMEM, std::string("ghost shell allocation failed: ") + hipGetErrorString(e));
            }
        }
    }
    hier_geometry(H);
    // scratch of the separable prolongation: two levels of every patch of
    // the depth that needs most (a window's extent does not depend on where
    // the patch sits); a third level after a move goes into a later batch
    size_t nx = 0, ny = 0;
    for (int d = 1; d < (int)H->dp.size(); ++d) {
        size_t sx = 0, sy = 0;
        for (int l : H->dp[d].q) {
            const HierPatch& P = H->pt[l];
            int Y0, NY, Z0, NZ;
            sep_window(P.L, P.plane, Y0, NY, Z0, NZ);
            const size_t NCx = P.L.n[0] + 2 * P.L.ng, NCy = P.L.n[1] + 2 * P.L.ng;
            sx += 2 * (size_t)NF * NZ * NY * NCx;
            sy += 2 * (size_t)NF * NZ * NCy * NCx;
        }
        nx = std::max(nx, sx);
        ny = std::max(ny, sy);
    }
    H->sepx_cap = nx;
    H->sepy_cap = ny;
    if (nx) {
        hipError_t e = hipMalloc((void**)&H->sepx, nx * sizeof(double));
        if (e != hipSuccess) H->sepx = nullptr;
        if (H->sepx && (e = hipMalloc((void**)&H->sepy, ny * sizeof(double))) != hipSuccess) H->sepy = nullptr;
        if (!H->sepx || !H->sepy) {
            hier_free(H);
            return fail(Z4C_ENOMEM, std::string("prolongation scratch allocation failed: ") + hipGetErrorString(e));
        }
    }
    for (int d = 0; d < (int)H->dp.size(); ++d) hier_build_sets(H, d);
    *hier = H;
    return Z4C_OK;
}

// capture one root step on the private stream (every parent holds an
// earlier level, so the schedule no longer changes from step to step)
static int hier_capture(z4c_hier_s* H)
{
    hipError_t e;
    if (!H->capture && (e = hipStreamCreateWithFlags(&H->capture, hipStreamNonBlocking)) != hipSuccess) {
        H->capture = nullptr;
        return hip_fail(e, "hipStreamCreateWithFlags");
    }
    // captured on a private stream; the instantiated graph runs on the caller's
    if ((e = hipStreamBeginCapture(H->capture, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = hier_depth_step(H, 0, 0.0, H->capture);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(H->capture, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "hierarchy step launch during capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    H->graph = g;
    H->exec = x;
    return Z4C_OK;
}

// After a root step: read the punctures back and shift every moving patch
// (in index order, so parents first) whose centre is more than two of its
// cells away from its object's puncture (per direction) by two cells toward
// it; cells it covered before keep their values, new ones are prolonged from
// the (already shifted) parent, and its children keep their place in space.
// The captured step is dropped when a patch moved (its geometry is baked
// into the graph).
static int hier_regrid(z4c_hier_s* H, hipStream_t s)
{
    hipError_t e;
    std::vector<double> st(10 * (size_t)H->nobj);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if ((e = hipMemcpy(st.data(), H->track, st.size() * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "hipMemcpy (punctures)");
    for (int o = 0; o < H->nobj; ++o)
        if (st[10 * o + 9] != 0.0)
            return fail(Z4C_EINVAL, "puncture " + std::to_string(o) + " left the active cells of its finest patch");
    const int np = (int)H->pt.size();
    bool moved = false;
    // whatever happens below, patches that did move must not run on launch
    // sets and a captured graph of their old geometry
    auto finish = [&](int rc) {
        if (moved) {
            for (int d = 0; d < (int)H->dp.size(); ++d) hier_build_sets(H, d);
            hier_drop_graph(H);
        }
        return rc;
    };
    for (int q = 1; q < np; ++q) {
        HierPatch& P = H->pt[q];
        const int o = P.L.obj;
        if (o < 0 || o >= H->nobj) continue;
        int sh[3];
        bool any = false;
        for (int d = 0; d < 3; ++d) {
            const double c = P.L.x0[d] + 0.5 * (P.L.n[d] - 1) * P.L.dx[d];
            const double x = st[10 * o + d];
            sh[d] = x - c > 2.0 * P.L.dx[d] ? 1 : (x - c < -2.0 * P.L.dx[d] ? -1 : 0);
            if (d == 2 && P.plane) sh[d] = 0;  // a patch on the symmetry plane stays on it
            any |= sh[d] != 0;
        }
        if (!any) continue;
        z4c_level nl = P.L;
        for (int d = 0; d < 3; ++d) {
            nl.F[d] += sh[d];
            nl.x0[d] += 2.0 * sh[d] * P.L.dx[d];
        }
        int rc;
        const std::string tag = "regrid of patch " + std::to_string(q) + ": ";
        const HierPatch& R = H->pt[P.L.parent];
        if ((rc = hier_check_level(nl, R.L, P.plane, tag))) return finish(rc);
        for (int c = q + 1; c < np; ++c) {
            if (H->pt[c].L.parent != q) continue;
            z4c_level cl = H->pt[c].L;
            for (int d = 0; d < 3; ++d) cl.F[d] -= 2 * sh[d];
            if ((rc = hier_check_level(cl, nl, H->pt[c].plane, tag + "child " + std::to_string(c) + ": ")))
                return finish(rc);
        }
        ShiftArgs a{};
        a.uc = P.L.u;
        a.out = P.L.u_a;
        a.sfc = P.L.sf;
        a.ngc = P.L.ng;
        a.up = R.L.u;
        a.sfp = R.L.sf;
        a.ngp = R.L.ng;
        for (int d = 0; d < 3; ++d) {
            a.Nc[d] = P.L.n[d] + 2 * P.L.ng;
            a.nc[d] = P.L.n[d];
            a.s[d] = sh[d];
            a.Np[d] = R.L.n[d] + 2 * R.L.ng;
            a.F[d] = nl.F[d];
        }
        a.refl = P.plane ? 1 : 0;
        if ((e = launch_shift(a, s)) != hipSuccess) return finish(hip_fail(e, "patch shift launch"));
        if ((e = launch_copy(P.L.u, P.L.u_a, (long)NF * P.L.sf, s)) != hipSuccess)
            return finish(hip_fail(e, "copy launch"));
        P.L = nl;
        P.has_prev = false;
        P.lev_cur = false;  // its ghosts sit elsewhere now
        for (int c = q + 1; c < np; ++c)
            if (H->pt[c].L.parent == q) {
                for (int d = 0; d < 3; ++d) H->pt[c].L.F[d] -= 2 * sh[d];
                H->pt[c].lev_cur = false;
            }
        hier_geometry(H);
        moved = true;
    }
    return finish(Z4C_OK);
}

int z4c_hier_advance(void* hier, int nsteps, int use_graph, void* stream)
{
    if (!hier) return fail(Z4C_EINVAL, "hier is NULL");
    if (nsteps < 0) return fail(Z4C_EINVAL, "nsteps must be >= 0");
    z4c_hier_s* H = (z4c_hier_s*)hier;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pending HIP error before z4c_hier_advance");
    auto primed = [&]() {
        const int last = (int)H->dp.size() - 1;
        for (const HierPatch& P : H->pt)
            if (P.depth < last && !P.has_prev) return false;
        return true;
    };
    for (int i = 0; i < nsteps; ++i) {
        // until every parent holds an earlier level the schedule changes from
        // step to step: those steps are launched directly
        if (use_graph && primed()) {
            int rc;
            if (!H->exec && (rc = hier_capture(H))) return rc;
            if ((e = hipGraphLaunch(H->exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        } else if ((e = hier_depth_step(H, 0, 0.0, s)) != hipSuccess) {
            return hip_fail(e, "hierarchy step launch");
        }
        if (H->nobj > 0) {
            int rc = hier_regrid(H, s);
            if (rc) return rc;
        }
    }
    return Z4C_OK;
}

int z4c_hier_set_moving(void* hier, int nobj, const double* xp)
{
    if (!hier || !xp) return fail(Z4C_EINVAL, "hier and xp must be non-NULL");
    z4c_hier_s* H = (z4c_hier_s*)hier;
    if (nobj < 1 || nobj > MAXEX) return fail(Z4C_EINVAL, "nobj must be 1..16");
    for (int i = 0; i < 3 * nobj; ++i)
        if (!std::isfinite(xp[i])) return fail(Z4C_EINVAL, "non-finite puncture position");
    int tp[MAXEX];
    for (int o = 0; o < nobj; ++o) {
        int best = -1, count = 0;
        for (int q = 0; q < (int)H->pt.size(); ++q) {
            if (H->pt[q].L.obj != o) continue;
            if (best < 0 || H->pt[q].depth > H->pt[best].depth) {
                best = q;
                count = 1;
            } else if (H->pt[q].depth == H->pt[best].depth) {
                ++count;
            }
        }
        if (best < 0) return fail(Z4C_EINVAL, "object " + std::to_string(o) + " has no patch");
        if (count != 1) return fail(Z4C_EINVAL, "object " + std::to_string(o) + " has several patches at its deepest depth");
        tp[o] = best;
    }
    for (const HierPatch& P : H->pt)
        if (P.L.obj >= nobj) return fail(Z4C_EINVAL, "a patch follows an object index >= nobj");
    hipError_t e;
    if (nobj > H->nobj || !H->track) {
        if (H->track) (void)hipFree(H->track);
        H->track = nullptr;
        if ((e = hipMalloc((void**)&H->track, 80 * (size_t)nobj)) != hipSuccess) {
            H->track = nullptr;
            H->nobj = 0;
            return fail(Z4C_ENOMEM, std::string("puncture state allocation failed: ") + hipGetErrorString(e));
        }
    }
    std::vector<double> st(10 * (size_t)nobj, 0.0);
    for (int o = 0; o < nobj; ++o)
        for (int d = 0; d < 3; ++d) st[10 * o + d] = st[10 * o + 6 + d] = xp[3 * o + d];
    if ((e = hipMemcpy(H->track, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy (punctures)");
    H->nobj = nobj;
    for (int o = 0; o < nobj; ++o) H->tp[o] = tp[o];
    hier_drop_graph(H);
    return Z4C_OK;
}

int z4c_hier_puncture(void* hier, double* xp, int* F, double* x0)
{
    if (!hier) return fail(Z4C_EINVAL, "hier is NULL");
    z4c_hier_s* H = (z4c_hier_s*)hier;
    if (xp) {
        if (!H->track || H->nobj < 1) return fail(Z4C_EINVAL, "no moving patches (z4c_hier_set_moving)");
        std::vector<double> st(10 * (size_t)H->nobj);
        hipError_t e = hipMemcpy(st.data(), H->track, st.size() * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy (punctures)");
        for (int o = 0; o < H->nobj; ++o)
            for (int d = 0; d < 3; ++d) xp[3 * o + d] = st[10 * o + d];
    }
    for (size_t q = 0; q < H->pt.size(); ++q)
        for (int d = 0; d < 3; ++d) {
            if (F) F[3 * q + d] = H->pt[q].L.F[d];
            if (x0) x0[3 * q + d] = H->pt[q].L.x0[d];
        }
    return Z4C_OK;
}

int z4c_hier_destroy(void* hier)
{
    if (!hier) return fail(Z4C_EINVAL, "hier is NULL");
    hier_free((z4c_hier_s*)hier);
    return Z4C_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Constraint monitor without a caller workspace.  The block partial sums go
// to `scratch`, a fixed device array of this library: every device the
// library runs on holds its own copy until the process ends.  In host code
// `scratch` names a host-side stand-in, not device memory, so the kernels
// receive the device address that hipGetSymbolAddress returns for the
// current device, looked up once per device on its first call.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[Z4C_CONSTRAINTS_NOALLOC_MAX_BLOCKS * 4];

namespace {
constexpr int MAXDEV = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[MAXDEV] = {};
}  // namespace

extern "C" int z4c_constraints_noalloc(const double* u, double* c, double* norms, long sf, int nx, int ny, int nz,
                                       int ng, double dx, double dy, double dz, void* stream)
{
    long stored = 0;
    int rc;
    if ((rc = check_geom(sf, nx, ny, nz, ng, Z4C_BC_PERIODIC, &stored)) ||
        (rc = check_spacing(dx, dy, dz, 0.0, 0.0, 0.0)))
        return rc;
    if (!u || !norms) return fail(Z4C_EINVAL, "u and norms must be non-NULL");
    const int n[3] = {nx, ny, nz};
    const long nb = constraint_blocks(n);
    if (nb > Z4C_CONSTRAINTS_NOALLOC_MAX_BLOCKS)
        return fail(Z4C_EINVAL, "box too large for z4c_constraints_noalloc: " + std::to_string(nb) +
                                    " bricks of 8x8x4 cells, at most " +
                                    std::to_string((long)Z4C_CONSTRAINTS_NOALLOC_MAX_BLOCKS) +
                                    " (use z4c_constraints with a workspace)");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAXDEV) return fail(Z4C_EUNSUPPORTED, "device index beyond the library's table");
    double* ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_dev[dev]) {
            void* ptr = nullptr;
            if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess)
                return hip_fail(e, "hipGetSymbolAddress(scratch)");
            g_scratch_dev[dev] = (double*)ptr;
        }
        ws = g_scratch_dev[dev];
    }
    return constraints_impl(u, c, norms, ws, true, sf, nx, ny, nz, ng, dx, dy, dz, stream, "z4c_constraints_noalloc");
}
