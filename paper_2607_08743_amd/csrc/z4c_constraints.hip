// z4c_constraints.hip -- constraint monitor: Hamiltonian and momentum
// constraints of the vacuum 3+1 system on every active point, and their
// volume-normalised L2 norms (paper Sec. 2.3), with a reduction whose order is
// fixed by the launch shape (bitwise reproducible run to run).
//
//   H   = R - At_ij At^ij + (2/3) K^2,              K = Khat + 2 Theta
//   M^i = W^2 [ Dt_j At^ij - 3 At^ij d_j W / W - (2/3) gt^ij d_j K ]
// with R built exactly as in the right-hand side (evolved Gt in its d Gt
// term), Dt the covariant derivative of gt, and
//   d_j At^ij = gt^ia gt^jb d_j At_ab + At_ab d_j(gt^ia gt^jb),
//   d_j gt^ia = -gt^ic gt^ad d_j gt_cd.
// The derivative stencils are the 4th-order centred ones of the evolution.
// Fields are staged one at a time through LDS like in the fused kernel
// (16-byte LDS-DMA loads two fields ahead, or register loads for boxes whose
// rows are not 16-byte aligned).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "z4c_internal.h"

namespace z4c {

namespace {

// Brick of one block, one point per thread.  8x8x4 points (four waves) at
// two waves per SIMD let two blocks share a CU, so that one block's tile
// waits and barriers overlap the other's arithmetic.
constexpr int CX = 8, CY = 8, CZ = 4;
constexpr int CNT = CX * CY * CZ;

// Tile geometry.  The stencils reach 2 cells (centred first, second and
// mixed derivatives).  On the DMA path the x halo is 3 so that every tile row
// starts on an even element (16-byte loads); y and z keep the 2-cell halo.
template <bool DMA>
struct CTile {
    static constexpr int HX = DMA ? 3 : 2, H = 2;
    static constexpr int SX = CX + 2 * HX, SY = CY + 2 * H, SXY = SX * SY, TN = SXY * (CZ + 2 * H);
    static constexpr int NR = (TN / 2 + CNT - 1) / CNT;      // 16-byte rounds per thread (DMA)
    static constexpr int TNP = DMA ? NR * CNT * 2 : TN;       // padded tile
    static constexpr int NE = (TN + CNT - 1) / CNT;           // elements per thread (register path)
    static constexpr int NBUF = DMA ? 3 : 1;
};

__device__ __forceinline__ int sidx(int a, int b)
{
    return (a < b ? a : b) * (5 - (a < b ? a : b)) / 2 + (a < b ? b : a);
}

__device__ __forceinline__ void keep(double& x) { __asm__ volatile("" : "+v"(x)); }
// Re-define every element here (an empty asm that may change them): the
// arithmetic that follows cannot be hoisted above this point, which keeps
// the algebra in phases instead of one interleaved block that needs more
// registers than a wave has.
template <int N>
__device__ __forceinline__ void phase(double (&x)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) keep(x[i]);
}
template <int M, int N>
__device__ __forceinline__ void phase(double (&x)[M][N])
{
#pragma unroll
    for (int i = 0; i < M; ++i) phase(x[i]);
}

__device__ __forceinline__ double cd1(const double* t, int st, double i12h)
{
    return (8.0 * (t[st] - t[-st]) - (t[2 * st] - t[-2 * st])) * i12h;
}

__device__ __forceinline__ double cd2(const double* t, int st, double i12h2)
{
    const double c = t[0];
    return (16.0 * ((t[st] - c) + (t[-st] - c)) - ((t[2 * st] - c) + (t[-2 * st] - c))) * i12h2;
}

__device__ __forceinline__ double cmix(const double* t, int sa, int sb, double scale)
{
    auto g = [&](int o) { return 8.0 * (t[o + sb] - t[o - sb]) - (t[o + 2 * sb] - t[o - 2 * sb]); };
    return (8.0 * (g(sa) - g(-sa)) - (g(2 * sa) - g(-2 * sa))) * scale;
}

// Fields in staging order: gt (derivatives), Gt, W, Khat, Theta, At.
__device__ __forceinline__ int cseq(int i)
{
    return i < 6 ? F_GT + i : i < 9 ? F_GAM + (i - 6) : i == 9 ? F_W : i == 10 ? F_KH : i == 11 ? F_TH : F_AT + (i - 12);
}
constexpr int CNSEQ = 18;

// Every term is folded into the constraint it feeds as soon as its inputs
// exist, so that few values stay live across the staging sequence:
//   after gt:     the Christoffels (d gt dies), the Ricci terms quadratic in
//                 them and the connection terms of the covariant divergence
//                 in M^i (At at the point is loaded beside gt);
//   after W:      W^2 R_ij and its trace R (the Christoffels die here);
//   after Theta:  d K folded into gt^ij d_j K;
//   per At field: gt^ia gt^jb d_j At_ab.
template <bool DMA>
__global__ void __launch_bounds__(CNT) __attribute__((amdgpu_waves_per_eu(2, 8))) constraints_kernel(BoxSet set, double* c_out, double* partial)
{
    using T = CTile<DMA>;
    constexpr int SX = T::SX, SXY = T::SXY, TN = T::TN, TNP = T::TNP, NR = T::NR, NE = T::NE;
    // the block reduction reuses the tile buffers (4 sums per thread)
    constexpr int TILE_D = T::NBUF * TNP > 4 * CNT ? T::NBUF * TNP : 4 * CNT;
    __shared__ __attribute__((aligned(16))) double tiles[TILE_D];
    const BoxDev& B = set.box[0];
    const int tid = threadIdx.x;
    // Lane order.  A 64-bit LDS read serves 16 lanes (two 8-point rows) per
    // pass.  With the 14-double row pitch of the DMA tile, rows y and y+4 are
    // 448 bytes apart and fall in disjoint halves of the banks, so each wave
    // takes its rows in the order 0, 4, 1, 5, 2, 6, 3, 7 (the 12-double pitch
    // of the register tile keeps the plain order: y and y+1 overlap less there).
    const int q8 = (tid / CX) % CY;
    const int tx = tid % CX, ty = DMA ? (((q8 & 1) << 2) | (q8 >> 1)) : q8, tz = tid / (CX * CY);
    // Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b mod 8);
    // give each XCD one contiguous chunk of the brick sequence, so that bricks
    // that share halo rows are fetched through the same L2.  The grid is a
    // multiple of 8; blocks past the last brick have nothing to do.
    const long nbk = (long)B.nb[0] * B.nb[1] * B.nb[2];
    const long chunk = (long)gridDim.x / 8;
    const long w = (long)(blockIdx.x % 8) * chunk + blockIdx.x / 8;
    if (w >= nbk) return;  // the whole block: no barrier is left waiting
    // brick order x fastest, then z, then y: the resident blocks of an XCD
    // (two per CU) take whole x rows of consecutive z layers, so the z halos,
    // the largest part of a thin 8x8x4 brick's tile, are fetched through one L2
    const int bxi = (int)(w % B.nb[0]), bzi = (int)((w / B.nb[0]) % B.nb[2]), byi = (int)(w / ((long)B.nb[0] * B.nb[2]));
    const int ng = B.ng;
    const int Nx = B.n[0] + 2 * ng, Ny = B.n[1] + 2 * ng, Nz = B.n[2] + 2 * ng;
    const int i0 = bxi * CX, j0 = byi * CY, k0 = bzi * CZ;
    const bool valid = (i0 + tx < B.n[0]) && (j0 + ty < B.n[1]) && (k0 + tz < B.n[2]);
    const size_t sf = (size_t)B.sf;
    const size_t p = ((size_t)(k0 + tz + ng) * Ny + (j0 + ty + ng)) * Nx + (i0 + tx + ng);
    const int gx0 = i0 + ng - T::HX, gy0 = j0 + ng - T::H, gz0 = k0 + ng - T::H;
    const int cofs = (tz + T::H) * SXY + (ty + T::H) * SX + (tx + T::HX);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // the derivative factors are the same on every lane: scalar registers
    auto uni = [](double x) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(x);
        const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
        const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
        return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    };
    double i12h[3], i12h2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        i12h[d] = uni(1.0 / (12.0 * B.h[d]));
        i12h2[d] = uni(1.0 / (12.0 * B.h[d] * B.h[d]));
    }
    const double imix[3] = {uni(1.0 / (144.0 * B.h[0] * B.h[1])), uni(1.0 / (144.0 * B.h[0] * B.h[2])),
                            uni(1.0 / (144.0 * B.h[1] * B.h[2]))};

    // per-thread offsets of its tile slots in one field (element pairs on the
    // DMA path; slots outside the stored box read a harmless valid address
    // there and are filled with 0 on the register path)
    int off[DMA ? NR : NE];
#pragma unroll
    for (int r = 0; r < (DMA ? NR : NE); ++r) {
        const int e = DMA ? 2 * (r * CNT + tid) : tid + r * CNT;
        int o = DMA ? 0 : -1;
        if (e < TN) {
            const int lx = e % SX, ly = (e / SX) % T::SY, lz = e / SXY;
            const int gi = gx0 + lx, gj = gy0 + ly, gk = gz0 + lz;
            if (gi < Nx && gj < Ny && gk < Nz) o = (gk * Ny + gj) * Nx + gi;
        }
        off[r] = o;
    }
    auto tilebuf = [&](int k) -> double* {
        int o = k * TNP;
        __asm__ volatile("" : "+s"(o));
        return tiles + o;
    };
    auto dma_issue = [&](int f, int k) {
        const double* src = B.u_in + f * sf;
        double* dst = tilebuf(k) + 2 * 64 * wave;
#pragma unroll
        for (int r = 0; r < NR; ++r) lds_dma16(src + off[r], (lds_void*)(dst + 2 * CNT * r));
    };
    const double* t = tiles + cofs;
    // make element i of the sequence the staged field
    auto stage = [&](int i) {
        if constexpr (DMA) {
            if (i + 1 < CNSEQ)
                __builtin_amdgcn_s_waitcnt(VM_N(NR));
            else
                __builtin_amdgcn_s_waitcnt(VM_N(0));
            __builtin_amdgcn_s_waitcnt(LGKM0);
            bar();
            if (i + 2 < CNSEQ) dma_issue(cseq(i + 2), (i + 2) % 3);
            t = tilebuf(i % 3) + cofs;
        } else {
            const double* src = B.u_in + cseq(i) * sf;
            double v[NE];
#pragma unroll
            for (int r = 0; r < NE; ++r) v[r] = off[r] >= 0 ? src[off[r]] : 0.0;
            __syncthreads();
#pragma unroll
            for (int r = 0; r < NE; ++r)
                if (r + 1 < NE || tid + r * CNT < TN) tiles[tid + r * CNT] = v[r];
            __syncthreads();
        }
    };
    if constexpr (DMA) {
        dma_issue(cseq(0), 0);
        dma_issue(cseq(1), 1);
    }
    // (no pin on the gradient: the Hessian that follows it reuses its LDS
    // reads of the axis neighbours)
    auto grad = [&](double* d) {
        d[0] = cd1(t, 1, i12h[0]);
        d[1] = cd1(t, SX, i12h[1]);
        d[2] = cd1(t, SXY, i12h[2]);
    };
    // second derivatives; the memory clobbers keep the compiler from issuing
    // the LDS reads of all six at once (each read holds two registers until
    // it is used), which would exceed the register budget
    auto hess = [&](double* dd) {
        dd[0] = cd2(t, 1, i12h2[0]);
        dd[3] = cd2(t, SX, i12h2[1]);
        dd[5] = cd2(t, SXY, i12h2[2]);
        keep(dd[0]);
        keep(dd[3]);
        keep(dd[5]);
        __asm__ volatile("" ::: "memory");
        dd[1] = cmix(t, 1, SX, imix[0]);
        keep(dd[1]);
        __asm__ volatile("" ::: "memory");
        dd[2] = cmix(t, 1, SXY, imix[1]);
        keep(dd[2]);
        __asm__ volatile("" ::: "memory");
        dd[4] = cmix(t, SX, SXY, imix[2]);
        keep(dd[4]);
    };
    auto tr6 = [](const double* g, const double* x) {
        return g[0] * x[0] + g[3] * x[3] + g[5] * x[5] + 2.0 * (g[1] * x[1] + g[2] * x[2] + g[4] * x[4]);
    };

    // conformal metric and traceless curvature at the point (loaded after the
    // first tiles, so one round trip covers both); the flat state on idle lanes
    double gt[6], gu[6], At[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        gt[q] = valid ? B.u_in[(F_GT + q) * sf + p] : (q == 0 || q == 3 || q == 5 ? 1.0 : 0.0);
        At[q] = valid ? B.u_in[(F_AT + q) * sf + p] : 0.0;
    }
    {
        const double det = gt[0] * (gt[3] * gt[5] - gt[4] * gt[4]) - gt[1] * (gt[1] * gt[5] - gt[4] * gt[2])
                         + gt[2] * (gt[1] * gt[4] - gt[3] * gt[2]);
        const double id = 1.0 / det;
        gu[0] = (gt[3] * gt[5] - gt[4] * gt[4]) * id;
        gu[1] = (gt[2] * gt[4] - gt[1] * gt[5]) * id;
        gu[2] = (gt[1] * gt[4] - gt[2] * gt[3]) * id;
        gu[3] = (gt[0] * gt[5] - gt[2] * gt[2]) * id;
        gu[4] = (gt[2] * gt[1] - gt[0] * gt[4]) * id;
        gu[5] = (gt[0] * gt[3] - gt[1] * gt[1]) * id;
    }
    double Rt[6], C2[3][6], Auu[6], AA, Mp[3];
    {
        double dgt[6][3];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            stage(q);
            grad(dgt[q]);
            double dd[6];
            hess(dd);
            Rt[q] = -0.5 * tr6(gu, dd);
            keep(Rt[q]);
        }
        // Christoffel symbols (first kind C1, second kind C2); d gt dies here
        phase(dgt);
        phase(gu);
        double C1[3][6], Gtd[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = i; j < 3; ++j) {
                    C1[k][sidx(i, j)] = 0.5 * (dgt[sidx(k, j)][i] + dgt[sidx(k, i)][j] - dgt[sidx(i, j)][k]);
                    keep(C1[k][sidx(i, j)]);
                }
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                C2[k][q] = gu[sidx(k, 0)] * C1[0][q] + gu[sidx(k, 1)] * C1[1][q] + gu[sidx(k, 2)] * C1[2][q];
                keep(C2[k][q]);
            }
#pragma unroll
        for (int k = 0; k < 3; ++k) Gtd[k] = tr6(gu, C2[k]);
        phase(C1);
        phase(C2);
        phase(Gtd);
        // Ricci terms quadratic in the Christoffels:
        // gt^lm (Gamma^k_li Gamma_jkm + Gamma^k_lj Gamma_ikm + Gamma^k_im Gamma_klj) = M_ij + M_ji + T_ij
        // with Cu[a][b][l] = gt^lm Gamma_abm, M_ij = Gamma^k_li Cu[j][k][l], T_ij = Gamma^k_im Cu[k][j][m]
        double M[3][3], T3[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) M[i][j] = T3[i][j] = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b2 = 0; b2 < 3; ++b2) {
                double cu[3];
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    cu[l] = gu[sidx(l, 0)] * C1[a][sidx(b2, 0)] + gu[sidx(l, 1)] * C1[a][sidx(b2, 1)]
                          + gu[sidx(l, 2)] * C1[a][sidx(b2, 2)];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    M[i][a] += C2[b2][sidx(0, i)] * cu[0] + C2[b2][sidx(1, i)] * cu[1] + C2[b2][sidx(2, i)] * cu[2];
                    T3[i][b2] += C2[a][sidx(i, 0)] * cu[0] + C2[a][sidx(i, 1)] * cu[1] + C2[a][sidx(i, 2)] * cu[2];
                }
            }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                double s = M[i][j] + M[j][i] + T3[i][j];
#pragma unroll
                for (int k = 0; k < 3; ++k) s += 0.5 * Gtd[k] * (C1[i][sidx(j, k)] + C1[j][sidx(i, k)]);
                Rt[sidx(i, j)] += s;
                keep(Rt[sidx(i, j)]);
            }
        phase(C2);
        phase(At);
        phase(gu);
        // At^ij and At_ij At^ij; the connection terms of the covariant
        // divergence.  With D_j At^ij = gt^ia gt^jb D_j At_ab (the conformal
        // connection is metric compatible) and Am_c^j = gt^jb At_cb:
        //   D_j At^ij = gt^ia gt^jb d_j At_ab - gt^ia Gamma^c_ja Am_c^j - Gtd^c Am_c^i,
        // the first term summed per At component below.
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                double s = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b2 = 0; b2 < 3; ++b2) s += gu[sidx(i, a)] * gu[sidx(j, b2)] * At[sidx(a, b2)];
                Auu[sidx(i, j)] = s;
            }
        AA = tr6(Auu, At);
        double Am[3][3];  // Am[c][j] = gt^jb At_cb
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                Am[c][j] = gu[sidx(j, 0)] * At[sidx(c, 0)] + gu[sidx(j, 1)] * At[sidx(c, 1)] + gu[sidx(j, 2)] * At[sidx(c, 2)];
        double Tm[3];  // Gamma^c_ja Am_c^j
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int j = 0; j < 3; ++j) s += C2[c][sidx(j, a)] * Am[c][j];
            Tm[a] = s;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            Mp[i] = -(gu[sidx(i, 0)] * Tm[0] + gu[sidx(i, 1)] * Tm[1] + gu[sidx(i, 2)] * Tm[2])
                  - (Gtd[0] * Am[0][i] + Gtd[1] * Am[1][i] + Gtd[2] * Am[2][i]);
            keep(Mp[i]);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) keep(Auu[q]);
        keep(AA);
    }
    // evolved Gt in the Ricci tensor
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        stage(6 + a);
        double d[3];
        grad(d);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) Rt[sidx(i, j)] += 0.5 * (gt[sidx(a, i)] * d[j] + gt[sidx(a, j)] * d[i]);
#pragma unroll
        for (int q = 0; q < 6; ++q) keep(Rt[q]);
    }
    // conformal factor: W^2 R_ij and its trace (no division by W)
    double W, dW[3], R;
    {
        stage(9);
        W = t[0];
        grad(dW);
        double DDW[6];
        hess(DDW);
#pragma unroll
        for (int q = 0; q < 6; ++q) DDW[q] -= C2[0][q] * dW[0] + C2[1][q] * dW[1] + C2[2][q] * dW[2];
        const double trDDW = tr6(gu, DDW);
        double dW2 = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) dW2 += gu[sidx(i, j)] * dW[i] * dW[j];
        double W2R[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) W2R[q] = W * W * Rt[q] + W * (DDW[q] + gt[q] * trDDW) - 2.0 * gt[q] * dW2;
        R = tr6(gu, W2R);
        keep(R);
    }
    // trace of the extrinsic curvature: K and gt^ij d_j K
    double K, gk[3];
    {
        double dK[3];
        stage(10);
        K = t[0];
        grad(dK);
        stage(11);
        K += 2.0 * t[0];
        double d[3];
        grad(d);
#pragma unroll
        for (int c = 0; c < 3; ++c) dK[c] += 2.0 * d[c];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            gk[a] = gu[sidx(a, 0)] * dK[0] + gu[sidx(a, 1)] * dK[1] + gu[sidx(a, 2)] * dK[2];
            keep(gk[a]);
        }
    }
    // traceless curvature: gt^ia gt^jb d_j At_ab, one component at a time
    double div[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        stage(12 + q);
        double d[3];
        grad(d);
        // component q = (c, e) stands for At_ce and At_ec
        const int c = q < 3 ? 0 : (q < 5 ? 1 : 2);
        const int e = q < 3 ? q : (q < 5 ? q - 2 : 2);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double wgt = gu[sidx(a, c)] * gu[sidx(j, e)];
                if (c != e) wgt += gu[sidx(a, e)] * gu[sidx(j, c)];
                s += wgt * d[j];
            }
            div[a] += s;
            keep(div[a]);
        }
    }

    double cv[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
        cv[0] = R - AA + 2.0 * K * K / 3.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double aw = Auu[sidx(a, 0)] * dW[0] + Auu[sidx(a, 1)] * dW[1] + Auu[sidx(a, 2)] * dW[2];
            cv[1 + a] = W * W * (div[a] + Mp[a] - 3.0 * aw / W - 2.0 * gk[a] / 3.0);
        }
        if (c_out)
#pragma unroll
            for (int m = 0; m < 4; ++m) c_out[m * sf + p] = cv[m];
    }
    // fixed-order block reduction of C^2 in the (now free) tile buffers
    if constexpr (DMA) __builtin_amdgcn_s_waitcnt(VM_N(0));
    __syncthreads();
    double* red = tiles;
#pragma unroll
    for (int m = 0; m < 4; ++m) red[m * CNT + tid] = cv[m] * cv[m];
    __syncthreads();
    for (int s2 = CNT / 2; s2 > 0; s2 >>= 1) {
        if (tid < s2)
#pragma unroll
            for (int m = 0; m < 4; ++m) red[m * CNT + tid] += red[m * CNT + tid + s2];
        __syncthreads();
    }
    if (tid < 4) partial[w * 4 + tid] = red[tid * CNT];
}

// one block: fixed-order sum of the partial records (four values each), then
// the norms.  A single block keeps the order fixed; 1024 threads with four
// independent records in flight per thread keep enough loads outstanding to
// read a few MiB of partials at cache speed.
constexpr int NORM_T = 1024;
__global__ void __launch_bounds__(NORM_T) constraint_norms(const double* partial, long nrec, double inv_cells,
                                                           double* norms)
{
    __shared__ double red[4][NORM_T];
    const int tid = threadIdx.x;
    double s[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = 0; m < 4; ++m) s[j][m] = 0.0;
    long r = tid;
    for (; r + 3 * NORM_T < nrec; r += 4 * NORM_T) {
        double v[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int m = 0; m < 4; ++m) v[j][m] = partial[(r + j * NORM_T) * 4 + m];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int m = 0; m < 4; ++m) s[j][m] += v[j][m];
    }
    for (; r < nrec; r += NORM_T)
#pragma unroll
        for (int m = 0; m < 4; ++m) s[0][m] += partial[r * 4 + m];
#pragma unroll
    for (int m = 0; m < 4; ++m) red[m][tid] = (s[0][m] + s[1][m]) + (s[2][m] + s[3][m]);
    __syncthreads();
    for (int k = NORM_T / 2; k > 0; k >>= 1) {
        if (tid < k)
#pragma unroll
            for (int m = 0; m < 4; ++m) red[m][tid] += red[m][tid + k];
        __syncthreads();
    }
    if (tid < 4) norms[tid] = sqrt(red[tid][0] * inv_cells);
}

__global__ void __launch_bounds__(256) zero_fill(double* x, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

}  // namespace

long constraint_blocks(const int n[3])
{
    return (long)((n[0] + CX - 1) / CX) * ((n[1] + CY - 1) / CY) * ((n[2] + CZ - 1) / CZ);
}

hipError_t launch_norms(const double* partial, long n, double inv_cells, double* norms, hipStream_t s)
{
    hipLaunchKernelGGL(constraint_norms, dim3(1), dim3(NORM_T), 0, s, partial, n, inv_cells, norms);
    return hipGetLastError();
}

hipError_t launch_zero(double* x, long n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(zero_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

hipError_t launch_constraints(const BoxSet& set, double* c_out, double* norms, double* workspace, hipStream_t s)
{
    BoxSet one = set;
    BoxDev& B = one.box[0];
    B.nb[0] = (B.n[0] + CX - 1) / CX;
    B.nb[1] = (B.n[1] + CY - 1) / CY;
    B.nb[2] = (B.n[2] + CZ - 1) / CZ;
    const long nb = constraint_blocks(B.n);
    if (c_out) {
        const long n = 4 * B.sf;
        hipLaunchKernelGGL(zero_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c_out, n);
    }
    // 16-byte tile loads need tile rows on even elements of an aligned field
    const bool dma = B.ng % 2 == 1 && B.n[0] % 2 == 0 && B.sf % 2 == 0 && ((uintptr_t)B.u_in & 15) == 0;
    const unsigned grid = (unsigned)((nb + 7) / 8 * 8);  // whole XCD rounds
    if (dma)
        hipLaunchKernelGGL(constraints_kernel<true>, dim3(grid), dim3(CNT), 0, s, one, c_out, workspace);
    else
        hipLaunchKernelGGL(constraints_kernel<false>, dim3(grid), dim3(CNT), 0, s, one, c_out, workspace);
    const double cells = (double)B.n[0] * B.n[1] * B.n[2];
    hipLaunchKernelGGL(constraint_norms, dim3(1), dim3(NORM_T), 0, s, workspace, nb, 1.0 / cells, norms);
    return hipGetLastError();
}

}  // namespace z4c
