// z4c_hierarchy.hip -- inter-level transfers of the box-in-box hierarchy
// with Berger-Oliger time subcycling (paper Sec. 2.2.1): successive levels
// refine 2:1 on cell-centred grids, so every child cell centre sits a quarter
// parent cell from the centre of the parent cell that contains it.
//
//   prolongation: the child's ghost shell from one parent time level,
//     6th-order Lagrange interpolation in each direction (tensor product,
//     6x6x6 parent cells, in three separable passes); the ghost fill weights
//     the levels' shells per stage time;
//   restriction: every coarse cell covered by the active region of a finer
//     patch from the 4th-order Lagrange interpolation of the 4x4x4 child
//     cells around its centre (the mean where several patches cover it);
//   exchange between the patches of one depth: overlapping active cells take
//     their mean, a ghost inside another patch's active region its value;
//   moving patches: puncture tracking and two-cell patch shifts.
// All are HBM/L2 gather kernels, one thread per output point.
#include <hip/hip_runtime.h>

#include "z4c_internal.h"

namespace z4c {

namespace {

// Lagrange weight of node m among `count` consecutive integer nodes starting
// at `first`, at the point x (evaluated at compile time below)
constexpr double lagrange_weight(int first, int count, int m, double x)
{
    double num = 1.0, den = 1.0;
    for (int b = 0; b < count; ++b)
        if (b != m) {
            num *= x - double(first + b);
            den *= double(first + m) - double(first + b);
        }
    return num / den;
}

// 1-D prolongation weights.  A child cell in the upper half of its parent
// cell (offset +1/4) uses parent cells -2..+3 relative to the containing
// one, a child in the lower half (-1/4) the mirror image -3..+2.  Both are
// summed nearest node first (offsets s*{0, 1, -1, 2, -2, 3}, s = +-1) with
// the same weights, so that mirror-image child points add mirror-image
// terms in the same order and round identically (pi symmetry is kept bit
// for bit).
struct ProlongW {
    double w[6];  // weight of the node at offset kOff[m] (upper half)
};
__constant__ int kOff[6] = {0, 1, -1, 2, -2, 3};
constexpr ProlongW make_prolong_w()
{
    constexpr int off[6] = {0, 1, -1, 2, -2, 3};
    ProlongW w{};
    for (int m = 0; m < 6; ++m) w.w[m] = lagrange_weight(-2, 6, off[m] + 2, 0.25);
    return w;
}
__constant__ ProlongW kProlong = make_prolong_w();
// the same offsets and weights as compile-time constants (immediates in the
// separable passes)
constexpr int kOffC[6] = {0, 1, -1, 2, -2, 3};
constexpr ProlongW kProlongC = make_prolong_w();

// restriction: child centres at -3/2, -1/2, 1/2, 3/2 child cells from the
// parent centre, weights (r0, r1, r1, r0), summed as r1 (c1 + c2) + r0 (c0 + c3)
constexpr double kR0 = -1.0 / 16.0, kR1 = 9.0 / 16.0;
static_assert(lagrange_weight(-1, 4, 0, 0.5) == kR0 && lagrange_weight(-1, 4, 1, 0.5) == kR1,
              "4-point midpoint weights");

__device__ __forceinline__ void shell_index(long q, int nx, int ny, int nz, int ng, int& i, int& j, int& k)
{
    // every index here is below the stored points of one field (< 2^31):
    // 32-bit unsigned division is far cheaper than 64-bit
    const unsigned Nx = nx + 2 * ng, Ny = ny + 2 * ng;
    const unsigned A = Nx * Ny;
    const unsigned P = A - (unsigned)nx * ny;  // ghost points of a plane that crosses the active box
    const unsigned low = (unsigned)ng * A;
    unsigned u = (unsigned)q;
    if (u < low) {
        k = (int)(u / A);
        const unsigned r = u - (unsigned)k * A;
        j = (int)(r / Nx);
        i = (int)(r - (unsigned)j * Nx);
        return;
    }
    u -= low;
    if (u < (unsigned)nz * P) {
        const unsigned kk = u / P;
        k = ng + (int)kk;
        unsigned r = u - kk * P;
        const unsigned rows_lo = (unsigned)ng * Nx;
        if (r < rows_lo) {
            j = (int)(r / Nx);
            i = (int)(r - (unsigned)j * Nx);
            return;
        }
        r -= rows_lo;
        const unsigned w2 = 2 * ng;
        const unsigned mid = (unsigned)ny * w2;
        if (r < mid) {
            const unsigned jj = r / w2;
            j = ng + (int)jj;
            const int t = (int)(r - jj * w2);
            i = t < ng ? t : nx + t;
            return;
        }
        r -= mid;
        const unsigned jj = r / Nx;
        j = ng + ny + (int)jj;
        i = (int)(r - jj * Nx);
        return;
    }
    u -= (unsigned)nz * P;
    const unsigned kk = u / A;
    k = ng + nz + (int)kk;
    const unsigned r = u - kk * A;
    j = (int)(r / Nx);
    i = (int)(r - (unsigned)j * Nx);
}

// z parity of a field: -1 for the components with one z index
__device__ __forceinline__ double zpar(int f)
{
    return (f == F_GT + 2 || f == F_GT + 4 || f == F_AT + 2 || f == F_AT + 4 || f == F_GAM + 2 || f == F_BE + 2 ||
            f == F_BB + 2)
               ? -1.0
               : 1.0;
}

// stored z index of a parent layer, reflected across the symmetry plane
// (the lower face of the active cells) when refl and it lies below it
__device__ __forceinline__ int refl_layer(int kz, int ng, bool refl, bool& neg)
{
    neg = refl && kz < ng;
    return neg ? 2 * ng - 1 - kz : kz;
}

// child active index a -> parent active index of the containing cell and the
// side of it the child lies on (+1 upper half, -1 lower half)
__device__ __forceinline__ int prolong_cell(int a, int F, int& side)
{
    const int half = a >= 0 ? a / 2 : -((1 - a) / 2);  // floor(a / 2)
    side = (a - 2 * half) != 0 ? 1 : -1;
    return F + half;
}

// Field f of the parent levels pa (time weights wt) interpolated at the child
// point whose containing parent cell is (px, py, pz) (stored indices) and
// whose sides are (sx, sy, sz); refl: parent layers below the symmetry plane
// (stored z < ngp) are read as the mirror images of those above it.
__device__ __forceinline__ double prolong_value(const double* const pa[3], const double wt[3], long sfp, long Nx,
                                                long NxNy, int px, int py, int pz, int sx, int sy, int sz, int f,
                                                bool refl, int ngp)
{
    long ox[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) ox[m] = px + sx * kOff[m];
    const double par = zpar(f);
    double s = 0.0;
    for (int c = 0; c < 6; ++c) {
        bool neg;
        const long zc = (long)refl_layer(pz + sz * kOff[c], ngp, refl, neg) * NxNy;
        const double sg = neg ? par : 1.0;
        double syy = 0.0;
        for (int b = 0; b < 6; ++b) {
            const long row = f * sfp + zc + (long)(py + sy * kOff[b]) * Nx;
            double sxx = 0.0;
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                double v = 0.0;
                for (int t = 0; t < 3; ++t)
                    if (pa[t]) v += wt[t] * pa[t][row + ox[m]];
                sxx += kProlong.w[m] * v;
            }
            syy += kProlong.w[b] * sxx;
        }
        s += kProlong.w[c] * (sg * syy);
    }
    return s;
}

// Separable single-level prolongation, pass 1: x sums for every child x
// index and parent (y, z) row in the scratch window.
__device__ __forceinline__ bool in_rows(int r, const int f[4])
{
    return (r >= f[0] && r <= f[1]) || (r >= f[2] && r <= f[3]);
}

// Entry of a batch that the current block works on.  Entries start on
// block boundaries (begin: exclusive prefix sums of the entries' thread
// counts, each rounded up to whole blocks), so the entry is the same for the
// whole block and its fields are read with scalar loads.
__device__ __forceinline__ int block_entry(const long* begin, int n)
{
    const long g0 = (long)blockIdx.x * blockDim.x;
    int e = 0;
    while (e + 1 < n && g0 >= begin[e + 1]) ++e;
    return __builtin_amdgcn_readfirstlane(e);
}

// The three passes put the field in blockIdx.y; within a field every index
// is below the child's stored points (< 2^31), so it is split with 32-bit
// unsigned divisions.  The prefix sums of a batch count one field's threads.
__global__ void __launch_bounds__(256) sep_x(SepBatch b)
{
    const int ei = block_entry(b.bx, b.n);
    const SepArgs& a = b.e[ei];
    const int f = (int)blockIdx.y;
    const unsigned NCx = a.nc[0] + 2 * a.ngc, NY = a.NY;
    const unsigned l = (unsigned)((long)blockIdx.x * blockDim.x + threadIdx.x - b.bx[ei]);
    if (l >= (unsigned)a.NZ * NY * NCx) return;
    const unsigned row = l / NCx;  // rz * NY + sy
    const int i = (int)(l - row * NCx);
    const unsigned rz = row / NY;
    const int sy = (int)(row - rz * NY);
    // x sums that no y sum the ghosts need will read
    if (!(i < a.ngc || i >= a.nc[0] + a.ngc || in_rows(a.Z0 + (int)rz, a.zf) || in_rows(a.Y0 + sy, a.yf))) return;
    int sx;
    const int px = prolong_cell(i - a.ngc, a.F[0], sx) + a.ngp;
    const double* src = a.u + f * a.sfp + ((long)(a.Z0 + (int)rz + a.ngp) * a.Np[1] + (a.Y0 + sy + a.ngp)) * a.Np[0] + px;
    double sxx = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) sxx += kProlongC.w[m] * src[sx * kOffC[m]];
    a.X[(long)f * a.NZ * NY * NCx + l] = sxx;
}
__global__ void __launch_bounds__(256) sep_y(SepBatch b)
{
    const int ei = block_entry(b.by, b.n);
    const SepArgs& a = b.e[ei];
    const int f = (int)blockIdx.y;
    const unsigned NCx = a.nc[0] + 2 * a.ngc, NCy = a.nc[1] + 2 * a.ngc;
    const unsigned l = (unsigned)((long)blockIdx.x * blockDim.x + threadIdx.x - b.by[ei]);
    if (l >= (unsigned)a.NZ * NCy * NCx) return;
    const unsigned row = l / NCx;  // rz * NCy + j
    const int i = (int)(l - row * NCx);
    const unsigned rz = row / NCy;
    const int j = (int)(row - rz * NCy);
    // y sums of interior columns are needed only in the rows the z ghost layers read
    if (!(i < a.ngc || i >= a.nc[0] + a.ngc || j < a.ngc || j >= a.nc[1] + a.ngc || in_rows(a.Z0 + (int)rz, a.zf)))
        return;
    int sy;
    const int py = prolong_cell(j - a.ngc, a.F[1], sy) - a.Y0;
    const double* col = a.X + ((long)f * a.NZ + rz) * a.NY * NCx + i;
    double syy = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) syy += kProlongC.w[m] * col[(long)(py + sy * kOffC[m]) * NCx];
    a.Y[(long)f * a.NZ * NCy * NCx + l] = syy;
}
__global__ void __launch_bounds__(256) sep_z(SepBatch b)
{
    const int ei = block_entry(b.bz, b.n);
    const SepArgs& a = b.e[ei];
    const int f = (int)blockIdx.y;
    const long NCx = a.nc[0] + 2 * a.ngc, NCy = a.nc[1] + 2 * a.ngc;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x - b.bz[ei];
    if (q >= a.nshell) return;
    int i, j, k;
    shell_index(q, a.nc[0], a.nc[1], a.nc[2], a.ngc, i, j, k);
    int sz;
    const int pz = prolong_cell(k - a.ngc, a.F[2], sz);
    const double par = zpar(f);
    const double* base = a.Y + (long)f * a.NZ * NCy * NCx + (long)j * NCx + i;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        int r = pz + sz * kOffC[c];
        double sg = 1.0;
        if (a.refl && r < 0) {
            r = -1 - r;
            sg = par;
        }
        s += kProlongC.w[c] * (sg * base[(long)(r - a.Z0) * NCy * NCx]);
    }
    a.shell[f * a.nshell + q] = s;
}

// A moving patch shifted by 2 s of its cells (s per direction in -1..1):
// active cell a of the new patch is cell a + 2 s of the old one where that
// exists, else prolonged from the parent (one time level, new face index F).
__global__ void __launch_bounds__(256) shift_patch(ShiftArgs a)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long n0 = a.nc[0], n1 = a.nc[1];
    if (q >= n0 * n1 * a.nc[2]) return;
    const int i = (int)(q % n0), j = (int)((q / n0) % n1), k = (int)(q / (n0 * n1));
    const long Ncx = a.Nc[0], NcxNcy = (long)a.Nc[0] * a.Nc[1];
    const long dst = (long)(k + a.ngc) * NcxNcy + (long)(j + a.ngc) * Ncx + (i + a.ngc);
    const int si = i + 2 * a.s[0], sj = j + 2 * a.s[1], sk = k + 2 * a.s[2];
    if (si >= 0 && si < a.nc[0] && sj >= 0 && sj < a.nc[1] && sk >= 0 && sk < a.nc[2]) {
        const long src = (long)(sk + a.ngc) * NcxNcy + (long)(sj + a.ngc) * Ncx + (si + a.ngc);
        for (int f = 0; f < NF; ++f) a.out[f * a.sfc + dst] = a.uc[f * a.sfc + src];
        return;
    }
    int sx, sy, sz;
    const int px = prolong_cell(i, a.F[0], sx) + a.ngp;
    const int py = prolong_cell(j, a.F[1], sy) + a.ngp;
    const int pz = prolong_cell(k, a.F[2], sz) + a.ngp;
    const double* const pa[3] = {nullptr, a.up, nullptr};
    const double wt[3] = {0.0, 1.0, 0.0};
    const long Nx = a.Np[0], NxNy = (long)a.Np[0] * a.Np[1];
    for (int f = 0; f < NF; ++f)
        a.out[f * a.sfc + dst] = prolong_value(pa, wt, a.sfp, Nx, NxNy, px, py, pz, sx, sy, sz, f, a.refl != 0, a.ngp);
}

// Puncture tracking, dx/dt = -beta, Heun's method on the finest level's
// steps.  st = {x[3], b0[3], xs[3], err}.  mode 0 (before a step): b0 =
// beta(x), xs = x - dt b0; mode 1 (after it): x -= dt/2 (b0 + beta(xs)).
// beta by 4-point Lagrange interpolation in each direction (cell centres
// i0-1 .. i0+2 around the point, all active).  One thread: 64 terms per component.
__global__ void __launch_bounds__(64) track_puncture(TrackBatch batch)
{
    const TrackArgs& a = batch.a[blockIdx.x];
    // lane t loads stencil point (t & 3, (t >> 2) & 3, t >> 4) of the three
    // shift components (one round trip); lane 0 then sums them in index order
    __shared__ double val[3][64];
    const int t = threadIdx.x;
    double* st = a.state;
    const double* x = a.mode == 0 ? st : st + 6;
    double w[3][4];
    int lo[3];
    // every lane derives the same stencil from the same position
    for (int d = 0; d < 3; ++d) {
        const double sc = (x[d] - a.x0[d]) / a.h[d];
        const int n = a.N[d] - 2 * a.ng;
        // stencil cells i0-1 .. i0+2 must be active (with refl, z layers below
        // the symmetry plane are the mirror images of active ones): otherwise
        // flag it, read nothing
        const int reach = (d == 2 && a.refl) ? -n : 0;
        if (!(sc > -2.0 + reach && sc < n + 1.0)) {
            if (t == 0) st[9] = 1.0;
            return;
        }
        const int i0 = (int)floor(sc);
        if (i0 - 1 < reach || i0 + 2 >= n) {
            if (t == 0) st[9] = 1.0;
            return;
        }
        lo[d] = i0 - 1 + a.ng;
        const double r = sc - i0;
        // nodes -1, 0, 1, 2
        w[d][0] = (r - 0.0) * (r - 1.0) * (r - 2.0) / ((-1.0) * (-2.0) * (-3.0));
        w[d][1] = (r + 1.0) * (r - 1.0) * (r - 2.0) / ((1.0) * (-1.0) * (-2.0));
        w[d][2] = (r + 1.0) * (r - 0.0) * (r - 2.0) / ((2.0) * (1.0) * (-1.0));
        w[d][3] = (r + 1.0) * (r - 0.0) * (r - 1.0) / ((3.0) * (2.0) * (1.0));
    }
    const long Nx = a.N[0], NxNy = (long)a.N[0] * a.N[1];
    {
        const int i = t & 3, j = (t >> 2) & 3, k = t >> 4;
        bool neg;
        const int kz = refl_layer(lo[2] + k, a.ng, a.refl != 0, neg);
        const long p = (long)kz * NxNy + (long)(lo[1] + j) * Nx + (lo[0] + i);
        for (int c = 0; c < 3; ++c) val[c][t] = (neg ? zpar(F_BE + c) : 1.0) * a.u[(F_BE + c) * a.sf + p];
    }
    __syncthreads();
    if (t != 0) return;
    double b[3];
    for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k)
            for (int j = 0; j < 4; ++j)
                for (int i = 0; i < 4; ++i) s += w[2][k] * w[1][j] * w[0][i] * val[c][(k * 4 + j) * 4 + i];
        b[c] = s;
    }
    if (a.mode == 0) {
        for (int d = 0; d < 3; ++d) {
            st[3 + d] = b[d];
            st[6 + d] = st[d] - a.dt * b[d];
        }
    } else {
        for (int d = 0; d < 3; ++d) st[d] = st[d] - 0.5 * a.dt * (st[3 + d] + b[d]);
    }
}

// one direction of the restriction stencil, in the mirror-symmetric order
__device__ __forceinline__ double rsum(double c0, double c1, double c2, double c3)
{
    return kR1 * (c1 + c2) + kR0 * (c0 + c3);
}

__device__ __forceinline__ bool in_active(const PatchRef& p, int g0, int g1, int g2)
{
    const int a0 = g0 - p.off[0], a1 = g1 - p.off[1], a2 = g2 - p.off[2];
    return a0 >= 0 && a0 < p.n[0] && a1 >= 0 && a1 < p.n[1] && a2 >= 0 && a2 < p.n[2];
}

// stored index of lattice cell G in patch p
__device__ __forceinline__ long lattice_index(const PatchRef& p, int g0, int g1, int g2)
{
    return ((long)(g2 - p.off[2] + p.ng) * p.N[1] + (g1 - p.off[1] + p.ng)) * p.N[0] + (g0 - p.off[0] + p.ng);
}

// Every parent active cell covered by the active region of a patch of the
// finer depth takes that patch's restriction (the mean over the patches
// that cover it, summed in patch order).  One thread per (field, cell).
__global__ void __launch_bounds__(256) restrict_cover(RestrictArgs a)
{
    const long cells = (long)a.ext[0] * a.ext[1] * a.ext[2];
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long)NF * cells) return;
    const int f = (int)(g / cells);
    const long q = g - (long)f * cells;
    const PatchRef& P = a.parent;
    const int x = a.lo[0] + (int)(q % a.ext[0]);
    const int y = a.lo[1] + (int)((q / a.ext[0]) % a.ext[1]);
    const int z = a.lo[2] + (int)(q / ((long)a.ext[0] * a.ext[1]));
    const int G0 = P.off[0] + x, G1 = P.off[1] + y, G2 = P.off[2] + z;
    double s = 0.0;
    int cnt = 0;
    for (int c = 0; c < a.nchild; ++c) {
        const PatchRef& C = a.child[c];
        // the parent cell spans child cells ac, ac + 1 in each direction
        const int ac0 = 2 * G0 - C.off[0], ac1 = 2 * G1 - C.off[1], ac2 = 2 * G2 - C.off[2];
        if (ac0 < 0 || ac0 + 1 >= C.n[0] || ac1 < 0 || ac1 + 1 >= C.n[1] || ac2 < 0 || ac2 + 1 >= C.n[2]) continue;
        const long Ncx = C.N[0], NcxNcy = (long)C.N[0] * C.N[1];
        const double* u =
            C.u + f * C.sf + (long)(ac2 - 1 + C.ng) * NcxNcy + (long)(ac1 - 1 + C.ng) * Ncx + (ac0 - 1 + C.ng);
        double pl[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double rw[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double* row = u + k * NcxNcy + j * Ncx;
                rw[j] = rsum(row[0], row[1], row[2], row[3]);
            }
            pl[k] = rsum(rw[0], rw[1], rw[2], rw[3]);
        }
        const double v = rsum(pl[0], pl[1], pl[2], pl[3]);
        s = cnt ? s + v : v;
        ++cnt;
    }
    if (!cnt) return;
    const long pq = ((long)(z + P.ng) * P.N[1] + (y + P.ng)) * P.N[0] + (x + P.ng);
    P.u[f * P.sf + pq] = cnt == 1 ? s : s / cnt;
}

// Exchange at one depth, averaging: a lattice cell in the active regions of
// several patches takes their mean (summed in patch order) in all of them.
// The first patch holding the cell writes it, so each cell is written by one
// thread of one launch.
__global__ void __launch_bounds__(256) exchange_average(ExchArgs a)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)a.ext[0] * a.ext[1] * a.ext[2]) return;
    const int g0 = a.lo[0] + (int)(q % a.ext[0]);
    const int g1 = a.lo[1] + (int)((q / a.ext[0]) % a.ext[1]);
    const int g2 = a.lo[2] + (int)(q / ((long)a.ext[0] * a.ext[1]));
    int first = -1, cnt = 0;
    for (int b = 0; b < a.np; ++b)
        if (in_active(a.p[b], g0, g1, g2)) {
            if (first < 0) first = b;
            ++cnt;
        }
    if (first != a.t || cnt < 2) return;
    for (int f = 0; f < NF; ++f) {
        double s = 0.0;
        for (int b = 0; b < a.np; ++b)
            if (in_active(a.p[b], g0, g1, g2)) s += a.p[b].u[f * a.p[b].sf + lattice_index(a.p[b], g0, g1, g2)];
        const double v = s / cnt;
        for (int b = 0; b < a.np; ++b)
            if (in_active(a.p[b], g0, g1, g2)) a.p[b].u[f * a.p[b].sf + lattice_index(a.p[b], g0, g1, g2)] = v;
    }
}

// Exchange at one depth, ghosts: a ghost point of patch t that lies in the
// active region of another patch of the depth takes that patch's value (the
// first such patch in index order).  Only ghosts are written, only active
// cells are read.
__global__ void __launch_bounds__(256) exchange_ghosts(ExchArgs a)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)a.ext[0] * a.ext[1] * a.ext[2]) return;
    const int g0 = a.lo[0] + (int)(q % a.ext[0]);
    const int g1 = a.lo[1] + (int)((q / a.ext[0]) % a.ext[1]);
    const int g2 = a.lo[2] + (int)(q / ((long)a.ext[0] * a.ext[1]));
    const PatchRef& T = a.p[a.t];
    if (in_active(T, g0, g1, g2)) return;
    for (int b = 0; b < a.np; ++b) {
        if (b == a.t || !in_active(a.p[b], g0, g1, g2)) continue;
        const long src = lattice_index(a.p[b], g0, g1, g2), dst = lattice_index(T, g0, g1, g2);
        for (int f = 0; f < NF; ++f) T.u[f * T.sf + dst] = a.p[b].u[f * a.p[b].sf + src];
        return;
    }
}

__global__ void __launch_bounds__(256) copy_box(CopyBoxBatch b)
{
    const int ei = block_entry(b.begin, b.n);
    const CopyBoxArgs& a = b.e[ei];
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x - b.begin[ei];
    const long n = (long)a.ext[0] * a.ext[1] * a.ext[2];
    if (g >= (long)NF * n) return;
    const int f = (int)(g / n);
    const long r = g - (long)f * n;
    const int i = (int)(r % a.ext[0]);
    const int j = (int)((r / a.ext[0]) % a.ext[1]);
    const int k = (int)(r / ((long)a.ext[0] * a.ext[1]));
    const long p = f * a.sf + ((long)(a.lo[2] + k) * a.N[1] + (a.lo[1] + j)) * a.N[0] + (a.lo[0] + i);
    a.dst[p] = a.src[p];
}

__global__ void __launch_bounds__(256) copy_list(CopyList c)
{
    const int ei = block_entry(c.begin, c.n);
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x - c.begin[ei];
    if (i >= c.len[ei]) return;
    c.dst[ei][i] = c.src[ei][i];
}

__global__ void __launch_bounds__(256) copy_state(double* __restrict__ dst, const double* __restrict__ src, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

hipError_t launch_restrict(const RestrictArgs& a, hipStream_t s)
{
    const long n = (long)NF * a.ext[0] * a.ext[1] * a.ext[2];
    if (n <= 0 || a.nchild <= 0) return hipSuccess;
    hipLaunchKernelGGL(restrict_cover, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_exchange_average(const ExchArgs& a, hipStream_t s)
{
    const long n = (long)a.ext[0] * a.ext[1] * a.ext[2];
    if (n <= 0 || a.np < 2) return hipSuccess;
    hipLaunchKernelGGL(exchange_average, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_exchange_ghosts(const ExchArgs& a, hipStream_t s)
{
    const long n = (long)a.ext[0] * a.ext[1] * a.ext[2];
    if (n <= 0 || a.np < 2) return hipSuccess;
    hipLaunchKernelGGL(exchange_ghosts, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

void sep_counts(const SepArgs& a, long& nx, long& ny, long& nz)
{
    const long NCx = a.nc[0] + 2 * a.ngc, NCy = a.nc[1] + 2 * a.ngc;
    nx = a.nshell > 0 ? (long)a.NZ * a.NY * NCx : 0;
    ny = a.nshell > 0 ? (long)a.NZ * NCy * NCx : 0;
    nz = a.nshell > 0 ? a.nshell : 0;
}

hipError_t launch_prolong_sep(const SepBatch& b, hipStream_t s)
{
    if (b.n <= 0 || b.bz[b.n] <= 0) return hipSuccess;
    hipLaunchKernelGGL(sep_x, dim3((unsigned)((b.bx[b.n] + 255) / 256), NF), dim3(256), 0, s, b);
    hipLaunchKernelGGL(sep_y, dim3((unsigned)((b.by[b.n] + 255) / 256), NF), dim3(256), 0, s, b);
    hipLaunchKernelGGL(sep_z, dim3((unsigned)((b.bz[b.n] + 255) / 256), NF), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_shift(const ShiftArgs& a, hipStream_t s)
{
    const long n = (long)a.nc[0] * a.nc[1] * a.nc[2];
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(shift_patch, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_track(const TrackBatch& b, hipStream_t s)
{
    if (b.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(track_puncture, dim3((unsigned)b.n), dim3(64), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_copy_box(const CopyBoxBatch& b, hipStream_t s)
{
    if (b.n <= 0 || b.begin[b.n] <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_box, dim3((unsigned)((b.begin[b.n] + 255) / 256)), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_copy_list(const CopyList& c, hipStream_t s)
{
    if (c.n <= 0 || c.begin[c.n] <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_list, dim3((unsigned)((c.begin[c.n] + 255) / 256)), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_state, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace z4c
