// z4c_hierarchy.hip -- inter-level transfers of the box-in-box hierarchy
// with Berger-Oliger time subcycling (paper Sec. 2.2.1): successive levels
// refine 2:1 on cell-centred grids, so every child cell centre sits a quarter
// parent cell from the centre of the parent cell that contains it.
//
//   prolongation: the child's ghost shell from the parent, 6th-order Lagrange
//     interpolation in each direction (tensor product, 6x6x6 parent cells), of
//     the parent time levels combined with the caller's time weights;
//   restriction: every parent cell covered by the child's active region from
//     the 4th-order Lagrange interpolation of the 4x4x4 child cells around
//     its centre.
// Both are HBM/L2 gather kernels, one thread per output point.
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

// 1-D prolongation weights: a child cell in the lower half of its parent cell
// (offset -1/4) uses parent cells -3..+2, one in the upper half (+1/4) cells
// -2..+3, relative to the containing parent cell.
struct ProlongW {
    double lo[6], hi[6];
};
constexpr ProlongW make_prolong_w()
{
    ProlongW w{};
    for (int m = 0; m < 6; ++m) {
        w.lo[m] = lagrange_weight(-3, 6, m, -0.25);
        w.hi[m] = lagrange_weight(-2, 6, m, 0.25);
    }
    return w;
}
__constant__ ProlongW kProlong = make_prolong_w();

// restriction: child centres at -3/2, -1/2, 1/2, 3/2 child cells from the parent centre
constexpr double kR0 = -1.0 / 16.0, kR1 = 9.0 / 16.0;
static_assert(lagrange_weight(-1, 4, 0, 0.5) == kR0 && lagrange_weight(-1, 4, 1, 0.5) == kR1,
              "4-point midpoint weights");

__device__ __forceinline__ void shell_index(long q, int nx, int ny, int nz, int ng, int& i, int& j, int& k)
{
    const int Nx = nx + 2 * ng, Ny = ny + 2 * ng;
    const long A = (long)Nx * Ny;
    const long P = A - (long)nx * ny;
    const long low = (long)ng * A;
    if (q < low) {
        k = (int)(q / A);
        j = (int)((q % A) / Nx);
        i = (int)(q % Nx);
        return;
    }
    q -= low;
    if (q < (long)nz * P) {
        k = ng + (int)(q / P);
        long r = q % P;
        const long rows_lo = (long)ng * Nx;
        if (r < rows_lo) {
            j = (int)(r / Nx);
            i = (int)(r % Nx);
            return;
        }
        r -= rows_lo;
        const long mid = (long)ny * 2 * ng;
        if (r < mid) {
            j = ng + (int)(r / (2 * ng));
            const int t = (int)(r % (2 * ng));
            i = t < ng ? t : nx + t;
            return;
        }
        r -= mid;
        j = ng + ny + (int)(r / Nx);
        i = (int)(r % Nx);
        return;
    }
    q -= (long)nz * P;
    k = ng + nz + (int)(q / A);
    j = (int)((q % A) / Nx);
    i = (int)(q % Nx);
}

// child active index a -> first parent active index of its 6-point stencil
// and which weight row applies
__device__ __forceinline__ int prolong_first(int a, int F, bool& upper)
{
    const int half = a >= 0 ? a / 2 : -((1 - a) / 2);  // floor(a / 2)
    upper = (a - 2 * half) != 0;
    return F + half + (upper ? -2 : -3);
}

__global__ void __launch_bounds__(256) prolong_shell(ProlongArgs a)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nshell) return;
    int i, j, k;
    shell_index(q, a.nc[0], a.nc[1], a.nc[2], a.ngc, i, j, k);
    bool ux, uy, uz;
    const int lx = prolong_first(i - a.ngc, a.F[0], ux) + a.ngp;
    const int ly = prolong_first(j - a.ngc, a.F[1], uy) + a.ngp;
    const int lz = prolong_first(k - a.ngc, a.F[2], uz) + a.ngp;
    const double* wx = ux ? kProlong.hi : kProlong.lo;
    const double* wy = uy ? kProlong.hi : kProlong.lo;
    const double* wz = uz ? kProlong.hi : kProlong.lo;
    const long Nx = a.Np[0], NxNy = (long)a.Np[0] * a.Np[1];
    const long base = lz * NxNy + (long)ly * Nx + lx;
    for (int f = 0; f < NF; ++f) {
        double s = 0.0;
        for (int c = 0; c < 6; ++c) {
            double sy = 0.0;
            for (int b = 0; b < 6; ++b) {
                const long row = f * a.sfp + base + c * NxNy + b * Nx;
                double sx = 0.0;
#pragma unroll
                for (int m = 0; m < 6; ++m) {
                    double v = 0.0;
                    for (int t = 0; t < 3; ++t)
                        if (a.pa[t]) v += a.wt[t] * a.pa[t][row + m];
                    sx += wx[m] * v;
                }
                sy += wy[b] * sx;
            }
            s += wz[c] * sy;
        }
        a.shell[f * a.nshell + q] = s;
    }
}

__global__ void __launch_bounds__(256) restrict_cover(RestrictArgs a)
{
    const int m0 = a.nc[0] / 2, m1 = a.nc[1] / 2, m2 = a.nc[2] / 2;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)m0 * m1 * m2) return;
    const int x = (int)(q % m0), y = (int)((q / m0) % m1), z = (int)(q / ((long)m0 * m1));
    const long Ncx = a.Nc[0], NcxNcy = (long)a.Nc[0] * a.Nc[1];
    const long cb = (long)(2 * z - 1 + a.ngc) * NcxNcy + (long)(2 * y - 1 + a.ngc) * Ncx + (2 * x - 1 + a.ngc);
    const long pq = ((long)(a.F[2] + z + a.ngp) * a.Np[1] + (a.F[1] + y + a.ngp)) * a.Np[0] + (a.F[0] + x + a.ngp);
    const double r[4] = {kR0, kR1, kR1, kR0};
    for (int f = 0; f < NF; ++f) {
        const double* u = a.uc + f * a.sfc + cb;
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double sy = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const double* row = u + c * NcxNcy + b * Ncx;
                sy += r[b] * (((r[0] * row[0] + r[1] * row[1]) + r[2] * row[2]) + r[3] * row[3]);
            }
            s += r[c] * sy;
        }
        a.up[f * a.sfp + pq] = s;
    }
}

__global__ void __launch_bounds__(256) copy_state(double* __restrict__ dst, const double* __restrict__ src, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

hipError_t launch_prolong(const ProlongArgs& a, hipStream_t s)
{
    if (a.nshell <= 0) return hipSuccess;
    hipLaunchKernelGGL(prolong_shell, dim3((unsigned)((a.nshell + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_restrict(const RestrictArgs& a, hipStream_t s)
{
    const long n = (long)(a.nc[0] / 2) * (a.nc[1] / 2) * (a.nc[2] / 2);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(restrict_cover, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_state, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace z4c
