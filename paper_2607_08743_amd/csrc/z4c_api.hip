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
    auto span = [](const void* p, uintptr_t bytes, const void* q, uintptr_t qbytes) {
        const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
        return a < b + qbytes && b < a + bytes;
    };
    const uintptr_t ub = (uintptr_t)sf * NF * 8, cb = (uintptr_t)sf * 4 * 8, wb = (uintptr_t)need * 8;
    if (c && span(c, cb, u, ub)) return fail(Z4C_EINVAL, "c overlaps u");
    if (span(ws, wb, u, ub) || (c && span(ws, wb, c, cb)) || span(ws, wb, norms, 32))
        return fail(Z4C_EINVAL, "ws overlaps another argument");
    if (span(norms, 32, u, ub) || (c && span(norms, 32, c, cb))) return fail(Z4C_EINVAL, "norms overlaps another argument");
    const int n[3] = {nx, ny, nz};
    const double h[3] = {dx, dy, dz}, o[3] = {0, 0, 0};
    BoxSet set{};
    set.nbox = 1;
    set.box[0] = make_box(n, ng, Z4C_BC_PERIODIC, sf, h, o, 1.0);
    set.box[0].u_in = u;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pending HIP error before z4c_constraints");
    if ((e = launch_constraints(set, c, norms, ws, (hipStream_t)stream)) != hipSuccess)
        return hip_fail(e, "z4c_constraints launch");
    return Z4C_OK;
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

int z4c_plan_create(const z4c_box* boxes, int nbox, const z4c_params* p, const z4c_tile* tile, void** plan)
{
    int rc;
    if (!plan) return fail(Z4C_EINVAL, "plan is NULL");
    *plan = nullptr;
    if ((rc = check_params(p))) return rc;
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
    int ti = tile ? find_tile(p->precision, tile) : default_tile_index(p->precision);
    if (ti < 0) return fail(Z4C_EUNSUPPORTED, "no compiled tile of that shape for this precision");
    z4c_plan_s* P = new (std::nothrow) z4c_plan_s();
    if (!P) return fail(Z4C_ENOMEM, "plan allocation failed");
    P->boxes.assign(boxes, boxes + nbox);
    P->prm = to_dev(p);
    P->precision = p->precision;
    P->tile_index = ti;
    P->persistent = tile ? (tile->persistent ? 1 : 0) : 1;
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

int z4c_plan_autotune(void* plan, int reps, void* stream, z4c_tile* best, float* ms)
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
    plan_drop_graph(P);
    plan_build_sets(P);
    if (best) {
        *best = tab[best_i].tile;
        best->persistent = best_p;
    }
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
struct HierLevel {
    z4c_level L;
    double* shell;  // device: ghost shell filled by prolongation (levels >= 1)
    long nshell;
    bool has_prev;  // prev holds this level one step earlier
    BoxSet fused[4];
    BoxSet fill[4];  // ghost fill of the stage inputs u, a, b, a
};

struct z4c_hier_s {
    std::vector<HierLevel> lv;
    ParamsDev prm;
    int precision;
    int tile_index;
    int persistent;
    double dt0;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t capture;
    int lmove;      // first moving level (0: none)
    double* track;  // device: puncture x[3], b0[3], xs[3], error flag
};

// Geometry of level x against its parent P: 2:1 spacing, lower faces on
// parent cell F, every ghost's prolongation stencil in P's active cells.
static int hier_check_level(const z4c_level& x, const z4c_level& P, const std::string& tag)
{
    for (int d = 0; d < 3; ++d) {
        if (x.n[d] % 2) return fail(Z4C_EINVAL, tag + "active extents must be even");
        if (x.dx[d] != 0.5 * P.dx[d]) return fail(Z4C_EINVAL, tag + "dx must be half the parent's");
        const double want = P.x0[d] + (x.F[d] - 0.25) * P.dx[d];
        if (std::fabs(x.x0[d] - want) > 1e-9 * P.dx[d])
            return fail(Z4C_EINVAL, tag + "x0 does not put the lower faces on parent cell F");
        // first / last parent cell read by the ghost stencils: floor(a/2) - 3 for
        // a = -ng, and floor(a/2) + 3 for a = n + ng - 1
        const int a_lo = -x.ng, a_hi = x.n[d] + x.ng - 1;
        const int lo = x.F[d] + (a_lo >= 0 ? a_lo / 2 : -((1 - a_lo) / 2)) - 3;
        const int hi = x.F[d] + a_hi / 2 + 3;
        if (lo < 0 || hi >= P.n[d]) return fail(Z4C_EINVAL, tag + "prolongation stencil leaves the parent's active cells");
    }
    return Z4C_OK;
}

// (Re)build the stage and ghost-fill sets of level l from its geometry.
static void hier_build_sets(z4c_hier_s* H, int l)
{
    const TileEntry* tab = nullptr;
    tile_table(&tab);
    HierLevel& L = H->lv[l];
    const double dt = H->dt0 / (double)(1L << l);
    double* ins[4] = {L.L.u, L.L.u_a, L.L.u_b, L.L.u_a};
    double* outs[4] = {L.L.u_a, L.L.u_b, L.L.u_a, L.L.u};
    for (int st = 0; st < 4; ++st) {
        BoxDev d = make_box(L.L.n, L.L.ng, L.L.bc, L.L.sf, L.L.dx, L.L.x0, dt);
        d.u_in = ins[st];
        d.u_n = L.L.u;
        d.acc = L.L.acc;
        d.u_out = outs[st];
        d.shell = L.shell;
        BoxSet& F = L.fused[st];
        F = BoxSet{};
        F.nbox = 1;
        F.box[0] = d;
        finalize_set(F, tab[H->tile_index].tile);
        L.fill[st] = F;
    }
}

static hipError_t hier_track(z4c_hier_s* H, int l, int mode, hipStream_t s)
{
    const HierLevel& L = H->lv[l];
    TrackArgs a{};
    a.state = H->track;
    a.u = L.L.u;
    a.sf = L.L.sf;
    for (int d = 0; d < 3; ++d) {
        a.N[d] = L.L.n[d] + 2 * L.L.ng;
        a.x0[d] = L.L.x0[d];
        a.h[d] = L.L.dx[d];
    }
    a.ng = L.L.ng;
    a.dt = H->dt0 / (double)(1L << l);
    a.mode = mode;
    return launch_track(a, s);
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

static hipError_t hier_prolong(z4c_hier_s* H, int l, double theta, hipStream_t s)
{
    HierLevel& C = H->lv[l];
    const HierLevel& P = H->lv[l - 1];
    ProlongArgs a{};
    hier_time_weights(theta, P.has_prev, a.wt);
    a.pa[0] = P.has_prev ? P.L.prev : nullptr;
    a.pa[1] = P.L.cur;
    a.pa[2] = P.L.u;
    a.sfp = P.L.sf;
    for (int d = 0; d < 3; ++d) {
        a.Np[d] = P.L.n[d] + 2 * P.L.ng;
        a.nc[d] = C.L.n[d];
        a.F[d] = C.L.F[d];
    }
    a.ngp = P.L.ng;
    a.shell = C.shell;
    a.nshell = C.nshell;
    a.ngc = C.L.ng;
    return launch_prolong(a, s);
}

static hipError_t hier_restrict(z4c_hier_s* H, int l, hipStream_t s)
{
    const HierLevel& C = H->lv[l];
    HierLevel& P = H->lv[l - 1];
    RestrictArgs a{};
    a.uc = C.L.u;
    a.sfc = C.L.sf;
    a.ngc = C.L.ng;
    a.up = P.L.u;
    a.sfp = P.L.sf;
    a.ngp = P.L.ng;
    for (int d = 0; d < 3; ++d) {
        a.Nc[d] = C.L.n[d] + 2 * C.L.ng;
        a.nc[d] = C.L.n[d];
        a.Np[d] = P.L.n[d] + 2 * P.L.ng;
        a.F[d] = C.L.F[d];
    }
    return launch_restrict(a, s);
}

// One RK4 step of level l starting at theta0 (fraction of the parent step),
// then, if it has a child, the child's two steps, its ghost fill at the end
// time and the restriction.  Stage inputs get their ghosts at the stage
// times theta0 + {0, 1/4, 1/4, 1/2}.
static hipError_t hier_level_step(z4c_hier_s* H, int l, double theta0, hipStream_t s)
{
    const TileEntry* tab = nullptr;
    tile_table(&tab);
    const TileEntry& T = tab[H->tile_index];
    HierLevel& L = H->lv[l];
    const int nlev = (int)H->lv.size();
    const bool outer = l == 0 && (L.L.bc == Z4C_BC_SOMMERFELD || L.L.bc == Z4C_BC_EQUATORIAL);
    const long n = (long)NF * L.L.sf;
    hipError_t e;
    auto fill = [&](int st) -> hipError_t {
        if (l == 0 && L.L.bc == Z4C_BC_SOMMERFELD) return hipSuccess;
        return launch_ghosts(L.fill[st], s);
    };
    auto stage = [&](int st) -> hipError_t {
        hipError_t r = T.launch(L.fused[st], H->prm, MODE_STAGE, st + 1, H->persistent, s);
        if (r == hipSuccess && outer) r = launch_sommerfeld(L.fused[st], H->prm, MODE_STAGE, st + 1, s);
        return r;
    };
    if (l > 0 && theta0 == 0.0 && (e = hier_prolong(H, l, 0.0, s)) != hipSuccess) return e;
    if ((e = fill(0)) != hipSuccess) return e;
    if (l + 1 < nlev && (e = launch_copy(L.L.cur, L.L.u, n, s)) != hipSuccess) return e;
    const bool track = H->lmove > 0 && l == nlev - 1;
    if (track && (e = hier_track(H, l, 0, s)) != hipSuccess) return e;
    if ((e = stage(0)) != hipSuccess) return e;
    if (l > 0 && (e = hier_prolong(H, l, theta0 + 0.25, s)) != hipSuccess) return e;
    if ((e = fill(1)) != hipSuccess || (e = stage(1)) != hipSuccess) return e;
    if ((e = fill(2)) != hipSuccess || (e = stage(2)) != hipSuccess) return e;
    if (l > 0 && (e = hier_prolong(H, l, theta0 + 0.5, s)) != hipSuccess) return e;
    if ((e = fill(3)) != hipSuccess || (e = stage(3)) != hipSuccess) return e;
    if (track && (e = hier_track(H, l, 1, s)) != hipSuccess) return e;
    if (l + 1 < nlev) {
        if ((e = hier_level_step(H, l + 1, 0.0, s)) != hipSuccess) return e;
        if ((e = hier_level_step(H, l + 1, 0.5, s)) != hipSuccess) return e;
        if ((e = hier_prolong(H, l + 1, 1.0, s)) != hipSuccess) return e;
        if ((e = launch_ghosts(H->lv[l + 1].fill[0], s)) != hipSuccess) return e;
        if ((e = hier_restrict(H, l + 1, s)) != hipSuccess) return e;
        if ((e = launch_copy(L.L.prev, L.L.cur, n, s)) != hipSuccess) return e;
        L.has_prev = true;
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
    for (HierLevel& L : H->lv)
        if (L.shell) (void)hipFree(L.shell);
    if (H->track) (void)hipFree(H->track);
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
    if (!levels || nlev < 1 || nlev > MAXBOX) return fail(Z4C_EINVAL, "need 1..16 levels");
    if (!finite_pos(dt0)) return fail(Z4C_EINVAL, "dt0 must be finite and > 0");
    for (int l = 0; l < nlev; ++l) {
        const z4c_level& x = levels[l];
        const std::string tag = "level " + std::to_string(l) + ": ";
        long stored = 0;
        if ((rc = check_geom(x.sf, x.n[0], x.n[1], x.n[2], x.ng, x.bc, &stored)) ||
            (rc = check_spacing(x.dx[0], x.dx[1], x.dx[2], x.x0[0], x.x0[1], x.x0[2])))
            return fail(rc, tag + z4c_last_error());
        const double* arr[6] = {x.u, x.u_a, x.u_b, x.acc, x.prev, x.cur};
        for (int i = 0; i < 6; ++i) {
            if (!arr[i]) return fail(Z4C_EINVAL, tag + "all six state arrays are required");
            for (int j = 0; j < i; ++j)
                if (overlap(arr[i], arr[j], x.sf)) return fail(Z4C_EINVAL, tag + "state arrays overlap");
        }
        if (l == 0) {
            if (x.bc == Z4C_BC_COPY) return fail(Z4C_EINVAL, tag + "the coarsest level needs its own boundary");
            continue;
        }
        if (x.bc != Z4C_BC_COPY) return fail(Z4C_EINVAL, tag + "levels >= 1 take Z4C_BC_COPY (filled from the parent)");
        if ((rc = hier_check_level(x, levels[l - 1], tag))) return rc;
    }
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
    const TileEntry* tab = nullptr;
    tile_table(&tab);
    z4c_hier_s* H = new z4c_hier_s{};
    H->prm = to_dev(p);
    H->precision = p->precision;
    H->tile_index = ti;
    H->persistent = pers;
    H->dt0 = dt0;
    H->lv.resize(nlev);
    for (int l = 0; l < nlev; ++l) {
        HierLevel& L = H->lv[l];
        L.L = levels[l];
        L.shell = nullptr;
        L.has_prev = false;
        L.nshell = l > 0 ? shell_size(L.L.n, L.L.ng) : 0;
        if (l > 0) {
            hipError_t e = hipMalloc((void**)&L.shell, (size_t)NF * L.nshell * sizeof(double));
            if (e != hipSuccess) {
                L.shell = nullptr;
                hier_free(H);
                return fail(Z4C_ENOMEM, "ghost shell allocation failed");
            }
        }
        hier_build_sets(H, l);
    }
    *hier = H;
    return Z4C_OK;
}

// capture one coarse step on the private stream (every parent holds an
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
    hipError_t le = hier_level_step(H, 0, 0.0, H->capture);
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

// After a coarse step: read the puncture back and shift every moving patch
// whose centre is more than two of its cells away from it (per direction)
// by two cells toward it; cells it covered before keep their values, new
// ones are prolonged from the (already shifted) parent.  The captured step
// is dropped when a patch moved (its geometry is baked into the graph).
static int hier_regrid(z4c_hier_s* H, hipStream_t s)
{
    hipError_t e;
    double st[10];
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if ((e = hipMemcpy(st, H->track, sizeof(st), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "hipMemcpy (puncture)");
    if (st[9] != 0.0) return fail(Z4C_EINVAL, "the puncture left the finest level");
    const int nlev = (int)H->lv.size();
    bool moved = false;
    for (int l = H->lmove; l < nlev; ++l) {
        HierLevel& L = H->lv[l];
        int sh[3];
        bool any = false;
        for (int d = 0; d < 3; ++d) {
            const double c = L.L.x0[d] + 0.5 * (L.L.n[d] - 1) * L.L.dx[d];
            sh[d] = st[d] - c > 2.0 * L.L.dx[d] ? 1 : (st[d] - c < -2.0 * L.L.dx[d] ? -1 : 0);
            any |= sh[d] != 0;
        }
        if (!any) continue;
        z4c_level nl = L.L;
        for (int d = 0; d < 3; ++d) {
            nl.F[d] += sh[d];
            nl.x0[d] += 2.0 * sh[d] * L.L.dx[d];
        }
        int rc;
        const std::string tag = "regrid of level " + std::to_string(l) + ": ";
        if ((rc = hier_check_level(nl, H->lv[l - 1].L, tag))) return rc;
        if (l + 1 < nlev) {
            z4c_level cl = H->lv[l + 1].L;
            for (int d = 0; d < 3; ++d) cl.F[d] -= 2 * sh[d];
            if ((rc = hier_check_level(cl, nl, tag + "child: "))) return rc;
        }
        const HierLevel& P = H->lv[l - 1];
        ShiftArgs a{};
        a.uc = L.L.u;
        a.out = L.L.u_a;
        a.sfc = L.L.sf;
        a.ngc = L.L.ng;
        a.up = P.L.u;
        a.sfp = P.L.sf;
        a.ngp = P.L.ng;
        for (int d = 0; d < 3; ++d) {
            a.Nc[d] = L.L.n[d] + 2 * L.L.ng;
            a.nc[d] = L.L.n[d];
            a.s[d] = sh[d];
            a.Np[d] = P.L.n[d] + 2 * P.L.ng;
            a.F[d] = nl.F[d];
        }
        if ((e = launch_shift(a, s)) != hipSuccess) return hip_fail(e, "patch shift launch");
        if ((e = launch_copy(L.L.u, L.L.u_a, (long)NF * L.L.sf, s)) != hipSuccess) return hip_fail(e, "copy launch");
        L.L = nl;
        L.has_prev = false;
        hier_build_sets(H, l);
        if (l + 1 < nlev)
            for (int d = 0; d < 3; ++d) H->lv[l + 1].L.F[d] -= 2 * sh[d];
        moved = true;
    }
    if (moved) hier_drop_graph(H);
    return Z4C_OK;
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
        for (size_t l = 0; l + 1 < H->lv.size(); ++l)
            if (!H->lv[l].has_prev) return false;
        return true;
    };
    for (int i = 0; i < nsteps; ++i) {
        // until every parent holds an earlier level the schedule changes from
        // step to step: those steps are launched directly
        if (use_graph && primed()) {
            int rc;
            if (!H->exec && (rc = hier_capture(H))) return rc;
            if ((e = hipGraphLaunch(H->exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        } else if ((e = hier_level_step(H, 0, 0.0, s)) != hipSuccess) {
            return hip_fail(e, "hierarchy step launch");
        }
        if (H->lmove > 0) {
            int rc = hier_regrid(H, s);
            if (rc) return rc;
        }
    }
    return Z4C_OK;
}

int z4c_hier_set_moving(void* hier, int lmove, const double* xp)
{
    if (!hier || !xp) return fail(Z4C_EINVAL, "hier and xp must be non-NULL");
    z4c_hier_s* H = (z4c_hier_s*)hier;
    const int nlev = (int)H->lv.size();
    if (lmove < 1 || lmove >= nlev) return fail(Z4C_EINVAL, "moving levels must start at 1..nlev-1");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(xp[d])) return fail(Z4C_EINVAL, "non-finite puncture position");
    hipError_t e;
    if (!H->track && (e = hipMalloc((void**)&H->track, 10 * sizeof(double))) != hipSuccess) {
        H->track = nullptr;
        return fail(Z4C_ENOMEM, "puncture state allocation failed");
    }
    const double st[10] = {xp[0], xp[1], xp[2], 0, 0, 0, xp[0], xp[1], xp[2], 0};
    if ((e = hipMemcpy(H->track, st, sizeof(st), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy (puncture)");
    H->lmove = lmove;
    hier_drop_graph(H);
    return Z4C_OK;
}

int z4c_hier_puncture(void* hier, double* xp, int* F, double* x0)
{
    if (!hier || !xp) return fail(Z4C_EINVAL, "hier and xp must be non-NULL");
    z4c_hier_s* H = (z4c_hier_s*)hier;
    if (!H->track) return fail(Z4C_EINVAL, "no moving levels (z4c_hier_set_moving)");
    double st[10];
    hipError_t e = hipMemcpy(st, H->track, sizeof(st), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy (puncture)");
    for (int d = 0; d < 3; ++d) xp[d] = st[d];
    for (size_t l = 0; l < H->lv.size(); ++l)
        for (int d = 0; d < 3; ++d) {
            if (F) F[3 * l + d] = H->lv[l].L.F[d];
            if (x0) x0[3 * l + d] = H->lv[l].L.x0[d];
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
