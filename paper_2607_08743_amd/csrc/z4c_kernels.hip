// z4c_kernels.hip -- gfx950 kernels of the fused Z4c right-hand side + RK4
// substep, the Sommerfeld ghost update and the periodic/copy ghost fill.
//
// Equations: the W-form Z4c system the paper adopts (arXiv 2607.08743,
// Sec. 2.1.1), with 1+log slicing and the Gamma-driver shift (Sec. 2.1.1
// gauge equations); 4th-order centred and shift-upwinded differences,
// 6th-order Kreiss-Oliger dissipation, classical RK4 (Sec. 2.2); the
// Sommerfeld outgoing condition (Sec. 2.2.2); det gt = 1 and tr At = 0
// restored after every substep (Sec. 2.1.1 states both hold).
//
// Fused kernel layout.  One thread owns one active point of a brick of
// BX*BY*BZ points.  The block stages the brick plus a 3-cell halo of ONE
// field at a time into LDS (the whole 25-field working set does not fit the
// 160 KB of LDS), and every thread folds that field's derivatives into
// running accumulators before the next field replaces it: second
// derivatives of gt go straight into the Ricci sum, those of beta into the
// Gt source, the advection + dissipation of every field into one scalar.
// Stencil reads are LDS reads at compile-time offsets.  After the last
// field the pointwise algebra, the RK4 update and the float64 enforcement
// run in registers and each thread writes its point once.  The path is a
// bandwidth/ALU-bound stencil, not a contraction: no MFMA.
//
// Precision.  R = double for Z4C_FP64.  For Z4C_MIXED R = float: the tiles
// are still float64 (DMA path) and every stencil difference is formed in
// float64 and then rounded to float32, so nearly-flat data keep their
// precision; the register path (boxes the DMA path cannot take) subtracts
// each field's flat value in float64 before the conversion.  k is promoted to
// float64 for the RK4 update and the enforcement.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "z4c_internal.h"

namespace z4c {

namespace {

// Materialise a value here: the empty volatile asm keeps the arithmetic that
// produces it on this side of the following barrier.  Without it the
// compiler sinks each staged field's stencil arithmetic to the end of the
// kernel, where the results are used, and keeps every loaded LDS value alive
// across all later barriers (hundreds of spilled registers).
template <typename R>
__device__ __forceinline__ void pin(R& x)
{
    __asm__ volatile("" : "+v"(x));
}
template <typename R, int N>
__device__ __forceinline__ void pin(R (&x)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) pin(x[i]);
}

// slot of the symmetric pair (a, b) in 6-component storage (xx xy xz yy yz zz);
// a closed form, so that it folds to a constant in every unrolled loop
__host__ __device__ constexpr int S(int a, int b)
{
    return (a < b ? a : b) * (5 - (a < b ? a : b)) / 2 + (a < b ? b : a);
}
static_assert(S(0, 0) == 0 && S(0, 1) == 1 && S(2, 0) == 2 && S(1, 1) == 3 && S(2, 1) == 4 && S(2, 2) == 5, "S");

__host__ __device__ constexpr double flat_of(int f)
{
    return (f == F_W || f == F_AL || f == F_GT + 0 || f == F_GT + 3 || f == F_GT + 5) ? 1.0 : 0.0;
}

// ------------------------------------------------------------------------
// LDS stencils.  `t` points at the thread's centre value in the staged tile,
// `st` is the stride of the direction (1, SX or SXY).  All one-direction
// operators are built from the even and odd differences
//     a_k = (f_k - f_0) + (f_-k - f_0),   b_k = f_k - f_-k,   k = 1, 2, 3
// (constant data give exact zeros; a pi-mirror pair of points gives exactly
// mirrored a, b):
//     D1  = (8 b1 - b2) / (12 h)            4th-order centred first derivative
//     D2  = (16 a1 - a2) / (12 h^2)         4th-order centred second derivative
//     KO6 = a3 - 6 a2 + 15 a1               sixth undivided difference
//     Dup = (O + s KO6) / (24 h),  O = 21 b1 - 6 b2 + b3,  s = sign(beta)
// The last line is an exact rewriting of the 5-point lopsided upwind stencil
// (-3, -10, 18, -6, 1)/(12 h) leaning toward s, so
//     beta Dup + sigma/(64 h) KO6 = beta/(24 h) O + (|beta|/(24 h) + sigma/(64 h)) KO6
// needs no per-lane select of the stencil direction.
// ------------------------------------------------------------------------
template <typename R>
struct Pairs {
    R a1, a2, a3, b1, b2, b3;
};

// the differences are formed in the tile's type TT and then rounded to R
template <typename R, typename TT>
__device__ __forceinline__ Pairs<R> pairs(const TT* t, int st)
{
    const TT c = t[0];
    const TT p1 = t[st], m1 = t[-st], p2 = t[2 * st], m2 = t[-2 * st], p3 = t[3 * st], m3 = t[-3 * st];
    Pairs<R> q;
    q.b1 = R(p1 - m1);
    q.b2 = R(p2 - m2);
    q.b3 = R(p3 - m3);
    q.a1 = R((p1 - c) + (m1 - c));
    q.a2 = R((p2 - c) + (m2 - c));
    q.a3 = R((p3 - c) + (m3 - c));
    return q;
}

template <typename R>
__device__ __forceinline__ R odd5(const Pairs<R>& q)
{
    return R(21) * q.b1 - R(6) * q.b2 + q.b3;
}

template <typename R>
__device__ __forceinline__ R ko6(const Pairs<R>& q)
{
    return (q.a3 - R(6) * q.a2) + R(15) * q.a1;
}

// A value known to be the same on every lane, moved to scalar registers.
__device__ __forceinline__ float uniform(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uniform(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// per-box derivative factors in the arithmetic type
template <typename R>
struct Factors {
    R i12h[3];   // 1/(12 h)
    R i12h2[3];  // 1/(12 h^2)
    R imix[3];   // 1/(144 h_a h_b) for (xy, xz, yz)
    R ko[3];     // sigma/(64 h)
    R i24h[3];   // 1/(24 h)
};

// 3x3 symmetric helpers on 6-component storage (xx xy xz yy yz zz)
template <typename T>
__device__ __forceinline__ T det6(const T* g)
{
    return g[0] * (g[3] * g[5] - g[4] * g[4]) - g[1] * (g[1] * g[5] - g[4] * g[2]) + g[2] * (g[1] * g[4] - g[3] * g[2]);
}

template <typename T>
__device__ __forceinline__ void inv6(const T* g, T* gi)
{
    const T id = T(1) / det6(g);
    gi[0] = (g[3] * g[5] - g[4] * g[4]) * id;
    gi[1] = (g[2] * g[4] - g[1] * g[5]) * id;
    gi[2] = (g[1] * g[4] - g[2] * g[3]) * id;
    gi[3] = (g[0] * g[5] - g[2] * g[2]) * id;
    gi[4] = (g[2] * g[1] - g[0] * g[4]) * id;
    gi[5] = (g[0] * g[3] - g[1] * g[1]) * id;
}

// contraction g^ij X_ij of two symmetric tensors
template <typename T>
__device__ __forceinline__ T tr6(const T* g, const T* x)
{
    return g[0] * x[0] + g[3] * x[3] + g[5] * x[5] + T(2) * (g[1] * x[1] + g[2] * x[2] + g[4] * x[4]);
}

// Restore det gt = 1 and tr At = 0 on one point (float64 in both precisions).
__device__ __forceinline__ void enforce(double* gt, double* At)
{
    const double s = 1.0 / cbrt(det6(gt));
#pragma unroll
    for (int q = 0; q < 6; ++q) gt[q] *= s;
    double gi[6];
    inv6(gt, gi);
    const double tr = tr6(gi, At) * (1.0 / 3.0);
#pragma unroll
    for (int q = 0; q < 6; ++q) At[q] -= gt[q] * tr;
}

// Write the RK4 stage (or the raw right-hand side) of one point of the fused
// kernel; kf(f) returns the right-hand side of field f.  Fields outside gt/At
// are stored as soon as they are updated; the 12 metric and curvature values
// wait for the enforcement.
template <typename KF>
__device__ __forceinline__ void finish_point(const BoxDev& B, int mode, int stage, KF kf, size_t p)
{
    const size_t sf = (size_t)B.sf;
    if (mode == MODE_RHS) {
#pragma unroll
        for (int f = 0; f < NF; ++f) B.u_out[f * sf + p] = kf(f);
        return;
    }
    const double dt = B.dt;
    const double c = stage == 3 ? dt : (stage == 4 ? dt / 6.0 : 0.5 * dt);
    // stage 1 and 4 update u_in and acc, stages 2 and 3 update u_n (and acc)
    const double* base = stage == 1 ? B.u_in : (stage == 4 ? B.acc : B.u_n);
    const bool upd = stage == 2 || stage == 3;
    // Every load is issued before the first is used (one round trip per
    // point; the caller has the registers to spare).  The empty asm keeps the
    // loads from being hoisted above this point, into code that has no
    // registers for them.
    double b0[NF], b1[NF];
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int f = 0; f < NF; ++f) b0[f] = base[f * sf + p];
    if (upd) {
#pragma unroll
        for (int f = 0; f < NF; ++f) b1[f] = B.acc[f * sf + p];
    }
    double gt[6], At[6];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const double k = kf(f);
        const double u0 = b0[f];
        const double v = u0 + c * k;
        if (stage == 1)
            B.acc[f * sf + p] = u0 + (dt / 6.0) * k;
        else if (upd)
            B.acc[f * sf + p] = b1[f] + (dt / 3.0) * k;
        if (f >= F_GT && f < F_GT + 6)
            gt[f - F_GT] = v;
        else if (f >= F_AT && f < F_AT + 6)
            At[f - F_AT] = v;
        else
            B.u_out[f * sf + p] = v;
    }
    enforce(gt, At);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        B.u_out[(F_GT + q) * sf + p] = gt[q];
        B.u_out[(F_AT + q) * sf + p] = At[q];
    }
}

// The stage update of finish_point for the Sommerfeld ghosts, over one of two
// field subsets: METRIC = gt and At (with the enforcement), else the 13
// others; loads five fields at a time (the empty asm keeps later fields' loads
// from being hoisted, which would cost registers this kernel's occupancy needs)
template <bool METRIC, typename KF>
__device__ __forceinline__ void finish_subset(const BoxDev& B, int mode, int stage, KF kf, size_t p)
{
    constexpr int NS = METRIC ? 12 : 13;
    auto fld = [](int r) {
        if (METRIC) return r < 6 ? F_GT + r : F_AT + (r - 6);
        return r == 0 ? F_W : r == 1 ? F_KH : r < 5 ? F_GAM + (r - 2) : r == 5 ? F_TH : r == 6 ? F_AL
             : r < 10 ? F_BE + (r - 7) : F_BB + (r - 10);
    };
    const size_t sf = (size_t)B.sf;
    if (mode == MODE_RHS) {
#pragma unroll
        for (int r = 0; r < NS; ++r) B.u_out[fld(r) * sf + p] = kf(fld(r));
        return;
    }
    const double dt = B.dt;
    const double c = stage == 3 ? dt : (stage == 4 ? dt / 6.0 : 0.5 * dt);
    const double* base = stage == 1 ? B.u_in : (stage == 4 ? B.acc : B.u_n);
    const bool upd = stage == 2 || stage == 3;
    double gt[6], At[6];
#pragma unroll
    for (int r = 0; r < NS; ++r) {
        if (r % 5 == 0) __asm__ volatile("" ::: "memory");
        const int f = fld(r);
        const double k = kf(f);
        const double u0 = base[f * sf + p];
        const double v = u0 + c * k;
        if (stage == 1)
            B.acc[f * sf + p] = u0 + (dt / 6.0) * k;
        else if (upd)
            B.acc[f * sf + p] = B.acc[f * sf + p] + (dt / 3.0) * k;
        if (METRIC) {
            if (r < 6)
                gt[r] = v;
            else
                At[r - 6] = v;
        } else {
            B.u_out[f * sf + p] = v;
        }
    }
    if constexpr (METRIC) {
        enforce(gt, At);
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            B.u_out[(F_GT + q) * sf + p] = gt[q];
            B.u_out[(F_AT + q) * sf + p] = At[q];
        }
    }
}

// ------------------------------------------------------------------------
// Fused right-hand side + RK4 substep over bricks of active points.
// ------------------------------------------------------------------------
template <typename R, int BX, int BY, int BZ>
struct Brick {
    static constexpr int NT = BX * BY * BZ;
    static constexpr int SX = BX + 6;
    static constexpr int SY = BY + 6;
    static constexpr int SXY = SX * SY;
    static constexpr int TN = SXY * (BZ + 6);
};

// Opaque copy of N values: arithmetic on it shares no subexpression with
// arithmetic on the originals.
template <typename R, int N>
struct MonCopy {
    R v[N];
    __device__ __forceinline__ explicit MonCopy(const R* x)
    {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            v[i] = x[i];
            pin(v[i]);
        }
    }
};

// Sum over the 64 lanes of a wave in a fixed butterfly order; every lane
// ends with a sum, lane 0's is returned in scalar registers (the lanes may
// round differently).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return uniform(v);
}

// MON: besides the stage, the constraint monitor of the stage input (Sec.
// 2.3): H and M^i at every active point (into mon.c when set) and, per wave
// of every brick, the sums of H^2 and (M^i)^2 over its points
// (mon.part[(brick * NT/64 + wave) * 4 + m]), from the same staged fields and
// derivatives as the right-hand side.
template <typename R, int BX, int BY, int BZ, int WAVES, bool DMA, bool MON = false>
__global__ void __attribute__((amdgpu_flat_work_group_size(BX* BY* BZ, BX* BY* BZ)))
__attribute__((amdgpu_waves_per_eu(WAVES, 8)))
fused_stage(BoxSet set, ParamsDev prm, int mode, int stage, MonDev mon)
{
    using T = Brick<R, BX, BY, BZ>;
    constexpr int NT = T::NT, SX = T::SX, SXY = T::SXY, TN = T::TN;
    static_assert(!DMA || (SX % 2 == 0 && NT % 64 == 0), "DMA staging: even rows, whole waves");
    // tile type: the DMA path stages float64 tiles in both precisions
    using TT = typename std::conditional<DMA, double, R>::type;
    // DMA staging moves pairs of doubles (16 bytes per lane); every wave issues
    // the same NR rounds, so the tile is padded to NR * NT pairs.
    constexpr int NR = (TN / 2 + NT - 1) / NT;
    constexpr int TNP = DMA ? NR * NT * 2 : TN;
    // Per-thread slots for values that are produced early and consumed late
    // (held advection terms, completed right-hand sides): parked in LDS
    // they take no registers across the staging sequence.  Slot s of thread
    // tid is park[s * NT + tid] (consecutive lanes, consecutive words).
    // The LDS share of one block (160 KB over the blocks a CU holds at WAVES
    // waves per SIMD) holds NBUF tile buffers -- the DMA path keeps NBUF - 1
    // fields in flight ahead of the one in use -- and the park slots; slots
    // beyond the share stay in registers.  One wave per SIMD has no other
    // wave to cover a late tile, so it gets as many buffers as fit next to all
    // 16 park slots (at most 7); two-wave shapes keep 3 so that their park
    // slots stay in LDS.
    constexpr int BPC = (WAVES * 4 * 64) / NT > 0 ? (WAVES * 4 * 64) / NT : 1;  // blocks per CU
    constexpr int BUDGET = 163840 / BPC - 512;
    constexpr int BUFB = (int)sizeof(TT) * TNP;
    constexpr int NB_FIT = (BUDGET - 16 * NT * (int)sizeof(R)) / BUFB;
    constexpr int NBUF = !DMA ? 1 : (WAVES > 1 || NB_FIT < 3) ? 3 : (NB_FIT > 7 ? 7 : NB_FIT);
    constexpr int DIST = NBUF - 1;  // fields in flight ahead of the staged one
    static_assert(!DMA || DIST * NR <= 63, "outstanding loads beyond the vmcnt range");
    constexpr int PARK_FIT = (BUDGET - NBUF * BUFB) / (NT * (int)sizeof(R));
    constexpr int NPARK = PARK_FIT < 0 ? 0 : (PARK_FIT > 16 ? 16 : PARK_FIT);
    __shared__ __attribute__((aligned(16))) TT tiles[NBUF * TNP];
    __shared__ __attribute__((aligned(16))) R park[(NPARK > 0 ? NPARK : 1) * NT];
    // MON: per-wave running sums of H^2 and (M^i)^2 over the bricks the wave
    // walks; only lane 0 of the wave reads or writes its four slots
    __shared__ double mon_acc[MON ? (NT / 64) * 4 : 1];
    // Buffer k of the tile.  The offset is made opaque to the compiler, so
    // that it adds it to the per-lane offsets when used instead of keeping
    // one precomputed address per buffer and lane offset live in registers.
    auto tilebuf = [&](int k) -> TT* {
        int o = k * TNP;
        __asm__ volatile("" : "+s"(o));
        return tiles + o;
    };

    const int tid = threadIdx.x;
    // Lane order.  A 64-bit LDS read serves 16 lanes per pass.  With 8-wide
    // bricks those are two rows of 8 points; rows y and y+4 sit 4 * 14 * 8
    // bytes apart, i.e. in disjoint halves of the 32 banks, so each wave's
    // rows are taken in the order 0, 4, 1, 5, 2, 6, 3, 7.
    const int q8 = (tid / BX) % BY;
    const int tx = tid % BX, ty = (BX == 8 && BY == 8) ? (((q8 & 1) << 2) | (q8 >> 1)) : q8, tz = tid / (BX * BY);
    const int cofs = (tz + 3) * SXY + (ty + 3) * SX + (tx + 3);
    const TT* tb = tiles;  // tile of the staged field
    const TT* t = tb + cofs;

    // Blocks are dealt to the 8 XCDs round-robin.  Give each XCD one
    // contiguous chunk of the brick sequence and let its resident blocks
    // walk it NS bricks at a time: bricks processed together, and in
    // consecutive rounds, are neighbours (x fastest, then y), so most of
    // their halos come from that XCD's L2.
    if constexpr (MON) {
        if ((tid & 63) == 0) {
#pragma unroll
            for (int m = 0; m < 4; ++m) mon_acc[(tid >> 6) * 4 + m] = 0.0;
        }
    }
    const long G = gridDim.x;
    const long b = blockIdx.x;
    const long total = set.brick_begin[set.nbox];
    const bool split = G % 8 == 0;
    const long NS = split ? G / 8 : G;              // blocks per XCD
    const long slot = split ? b / 8 : b;
    const long C = split ? (total + 7) / 8 : total;  // bricks per XCD
    const long first = (split ? (b % 8) * C : 0) + slot;
    const long last = split ? ((b % 8) + 1) * C < total ? ((b % 8) + 1) * C : total : total;

    for (long w = first; w < last; w += NS) {
        if (DMA && w != first) {
            // every wave is done with the previous brick's tiles before new loads land
            __builtin_amdgcn_s_waitcnt(LGKM0);
            bar();
        }
        int bi = 0;
        while (w >= set.brick_begin[bi + 1]) ++bi;
        const BoxDev& B = set.box[bi];
        const long lw = w - set.brick_begin[bi];
        const int bxi = (int)(lw % B.nb[0]);
        const int byi = (int)((lw / B.nb[0]) % B.nb[1]);
        const int bzi = (int)(lw / ((long)B.nb[0] * B.nb[1]));
        const int ng = B.ng;
        const int Nx = B.n[0] + 2 * ng, Ny = B.n[1] + 2 * ng, Nz = B.n[2] + 2 * ng;
        const int i0 = bxi * BX, j0 = byi * BY, k0 = bzi * BZ;  // active-relative brick origin
        const bool valid = (i0 + tx < B.n[0]) && (j0 + ty < B.n[1]) && (k0 + tz < B.n[2]);
        const size_t sf = (size_t)B.sf;
        const size_t p = ((size_t)(k0 + tz + ng) * Ny + (j0 + ty + ng)) * Nx + (i0 + tx + ng);
        // tile origin in stored coordinates (>= 0 because ng >= 3)
        const int gx0 = i0 + ng - 3, gy0 = j0 + ng - 3, gz0 = k0 + ng - 3;

        // the factors are the same on every lane: keep them in scalar registers
        Factors<R> fc;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            fc.i12h[d] = uniform(R(1.0 / (12.0 * B.h[d])));
            fc.i12h2[d] = uniform(R(1.0 / (12.0 * B.h[d] * B.h[d])));
            fc.ko[d] = uniform(R(prm.ko_sigma / (64.0 * B.h[d])));
            fc.i24h[d] = uniform(R(1.0 / (24.0 * B.h[d])));
        }
        fc.imix[0] = uniform(R(1.0 / (144.0 * B.h[0] * B.h[1])));
        fc.imix[1] = uniform(R(1.0 / (144.0 * B.h[0] * B.h[2])));
        fc.imix[2] = uniform(R(1.0 / (144.0 * B.h[1] * B.h[2])));

        // Field order of the staging sequence.
        constexpr int NSEQ = 25;
        auto seq = [](int i) -> int {
            return i < 6 ? F_GT + i
                 : i < 9 ? F_GAM + (i - 6)
                 : i == 9 ? F_W
                 : i == 10 ? F_AL
                 : i == 11 ? F_KH
                 : i == 12 ? F_TH
                 : i < 16 ? F_BE + (i - 13)
                 : i < 22 ? F_AT + (i - 16)
                 : F_BB + (i - 22);
        };

        // Register staging (float32 tiles, or boxes the DMA path does not take).
        // Each thread copies the same NE tile slots for every field; their
        // offsets inside a field (-1 outside the stored box) are computed once
        // per brick.  The next field is loaded into registers while the current
        // one is being differentiated, then written to the tile between two
        // barriers.
        constexpr int NE = DMA ? 1 : (TN + NT - 1) / NT;
        int goff[NE];
        double pre[NE];
        int pre_f = -1;
        // DMA staging (float64): each field's tile is loaded straight into one
        // of three LDS buffers two fields ahead of its use, without registers;
        // per round a wave moves 64 pairs of doubles into consecutive LDS.
        // Not every tile element is read.  The one-direction stencils (first,
        // second, upwind and dissipation differences) reach +-3 cells along
        // one axis; the mixed second derivatives of the 11 fields that need
        // them (gt, W, alpha, beta) also reach the edges of the tile with both
        // offsets <= 2.
        // Pairs outside that set (the tile's corners) are not fetched: their
        // lanes load the tile-centre pair instead, a line the same load
        // fetches anyway, so the corners cost no extra L2 or HBM traffic.
        // doff: offsets for the fields with mixed derivatives, doff1: for the
        // others (one-direction stencils only).
        int doff[DMA ? NR : 1], doff1[DMA ? NR : 1];
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        if constexpr (DMA) {
            const int oc = ((gz0 + 3 + BZ / 2) * Ny + (gy0 + 3 + BY / 2)) * Nx + (gx0 + 4);
            // distance of tile coordinate c outside the brick [3, 3 + Bn)
            auto outd = [](int c, int Bn) { return c < 3 ? 3 - c : (c >= 3 + Bn ? c - 2 - Bn : 0); };
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int e = 2 * (r * NT + tid);
                int o = 0;  // slots outside the stored box read a harmless valid address
                int o1 = 0;
                if (e < TN) {
                    const int lx = e % SX, ly = (e / SX) % T::SY, lz = e / SXY;
                    const int gi = gx0 + lx, gj = gy0 + ly, gk = gz0 + lz;
                    const int dx0 = outd(lx, BX), dx1 = outd(lx + 1, BX);
                    const int dx = dx0 < dx1 ? dx0 : dx1, dy = outd(ly, BY), dz = outd(lz, BZ);
                    const int nz = (dx > 0) + (dy > 0) + (dz > 0);
                    const bool need1 = nz <= 1;
                    const bool needm = need1 || (nz == 2 && dx <= 2 && dy <= 2 && dz <= 2);
                    if (gi < Nx && gj < Ny && gk < Nz) o = (gk * Ny + gj) * Nx + gi;
                    o1 = need1 ? o : oc;
                    if (!needm) o = oc;
                }
                doff[r] = o;
                doff1[r] = o1;
            }
        } else {
#pragma unroll
            for (int r = 0; r < NE; ++r) {
                const int e = tid + r * NT;
                int o = -1;
                if (e < TN) {
                    const int lx = e % SX, ly = (e / SX) % T::SY, lz = e / SXY;
                    const int gi = gx0 + lx, gj = gy0 + ly, gk = gz0 + lz;
                    if (gi < Nx && gj < Ny && gk < Nz) o = (gk * Ny + gj) * Nx + gi;
                }
                goff[r] = o;
            }
        }
        auto dma_issue = [&](int i, int k) {
            const double* src = B.u_in + seq(i) * sf;
            TT* dst = tilebuf(k) + 2 * 64 * wave;
            // sequence positions of gt, W, alpha and beta (the fields with mixed derivatives)
            const bool mixed = i < 6 || i == 9 || i == 10 || (i >= 13 && i < 16);
#pragma unroll
            for (int r = 0; r < NR; ++r) lds_dma16(src + (mixed ? doff[r] : doff1[r]), (lds_void*)(dst + 2 * NT * r));
        };
        auto prefetch = [&](int f) {
            const double* src = B.u_in + f * sf;
#pragma unroll
            for (int r = 0; r < NE; ++r) pre[r] = goff[r] >= 0 ? src[goff[r]] : 0.0;
            pre_f = f;
        };
        // wait until at most `later` fields' tile loads of this wave are in flight
        auto wait_fields = [&](int later) {
            if (later >= 6)
                __builtin_amdgcn_s_waitcnt(VM_N(6 * NR));
            else if (later == 5)
                __builtin_amdgcn_s_waitcnt(VM_N(5 * NR));
            else if (later == 4)
                __builtin_amdgcn_s_waitcnt(VM_N(4 * NR));
            else if (later == 3)
                __builtin_amdgcn_s_waitcnt(VM_N(3 * NR));
            else if (later == 2)
                __builtin_amdgcn_s_waitcnt(VM_N(2 * NR));
            else if (later == 1)
                __builtin_amdgcn_s_waitcnt(VM_N(NR));
            else
                __builtin_amdgcn_s_waitcnt(VM_N(0));
        };
        // make element i of the sequence the staged field
        auto stage_field = [&](int i) {
            if constexpr (DMA) {
                // wait until this wave's loads of field i have landed (those of
                // the later fields already issued may still be in flight), then
                // until every wave has, and has finished reading field i-1
                const int later = (NSEQ - 1 - i) < (DIST - 1) ? (NSEQ - 1 - i) : (DIST - 1);
                wait_fields(later);
                __builtin_amdgcn_s_waitcnt(LGKM0);
                bar();
                if (i + DIST < NSEQ) dma_issue(i + DIST, (i + DIST) % NBUF);
                tb = tilebuf(i % NBUF);
                t = tb + cofs;
            } else {
                const double off = sizeof(R) == 4 ? flat_of(pre_f) : 0.0;
                __syncthreads();
                TT* tw = tilebuf(0);
#pragma unroll
                for (int r = 0; r < NE; ++r) {
                    const int e = tid + r * NT;
                    if (r + 1 < NE || e < TN) tw[e] = goff[r] >= 0 ? R(pre[r] - off) : R(0);
                }
                __syncthreads();
                if (i + 1 < NSEQ) prefetch(seq(i + 1));
            }
        };
        if constexpr (DMA) {
#pragma unroll
            for (int k = 0; k < DIST; ++k) dma_issue(k, k);
        } else {
            prefetch(seq(0));
        }

        enum : int { P_AKGT = 0, P_AKGAM = 6, P_AKBE = 9, P_KKH = 12, P_KTH = 13, P_KAL = 14, P_KW = 15 };
        constexpr int P_AT0 = P_AKGAM;  // At at the point, until the Gt fields are staged (slots 6-11)
        R park_r[16];
        auto put_lds = [&](int slot, R v) {
            if (slot < NPARK)
                park[slot * NT + tid] = v;
            else
                park_r[slot] = v;
        };
        auto get_lds = [&](int slot) { return slot < NPARK ? park[slot * NT + tid] : park_r[slot]; };

        // Centre values needed before staging (the flat state on idle lanes
        // keeps the algebra finite); the others are taken from the tiles.
        // They are loaded after the first tiles' loads, so that waiting for
        // them (the compiler waits for all of its loads at their first use)
        // is one round trip for both.  At is needed after the metric; it is
        // parked in the slots that stay free until the Gt fields are staged.
        auto centre = [&](int f) { return valid ? R(B.u_in[f * sf + p]) : R(flat_of(f)); };
        R gt[6], gu[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) gt[q] = centre(F_GT + q);
        const R be[3] = {centre(F_BE), centre(F_BE + 1), centre(F_BE + 2)};
        {
            R At0[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) At0[q] = centre(F_AT + q);
#pragma unroll
            for (int q = 0; q < 6; ++q) put_lds(P_AT0 + q, At0[q]);
        }
        inv6(gt, gu);
        // advection + dissipation weights of the odd (O) and even (KO6) parts, per direction
        R wodd[3], wev[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            wodd[d] = be[d] * fc.i24h[d];
            wev[d] = (be[d] < R(0) ? -be[d] : be[d]) * fc.i24h[d] + fc.ko[d];
        }


        // centre value of the staged field (its flat value restored when the
        // register path staged it in float32)
        auto tval = [&](int f) {
            R v = R(t[0]) + R((sizeof(R) == 4 && !DMA) ? flat_of(f) : 0.0);
            pin(v);
            return v;
        };
        // even/odd differences of the staged field in the three directions
        struct P3 {
            Pairs<R> x, y, z;
        };
        auto field_pairs = [&]() { return P3{pairs<R>(t, 1), pairs<R>(t, SX), pairs<R>(t, SXY)}; };
        // advection along the shift plus Kreiss-Oliger dissipation
        auto advko = [&](const P3& q) {
            R a = (wodd[0] * odd5(q.x) + wev[0] * ko6(q.x)) + (wodd[1] * odd5(q.y) + wev[1] * ko6(q.y))
                + (wodd[2] * odd5(q.z) + wev[2] * ko6(q.z));
            pin(a);
            return a;
        };
        auto grad = [&](const P3& q, R* d) {
            d[0] = (R(8) * q.x.b1 - q.x.b2) * fc.i12h[0];
            d[1] = (R(8) * q.y.b1 - q.y.b2) * fc.i12h[1];
            d[2] = (R(8) * q.z.b1 - q.z.b2) * fc.i12h[2];
        };
        // Mixed second difference of the staged field straight from the tile:
        // the 4th-order first difference along sa of the 4th-order first
        // difference along sb (16 LDS reads, unscaled).  No intermediate
        // plane, so no barrier between filling and reading one.
        auto mixd = [&](int sa, int sb) {
            auto u1 = [&](int c) { return R(TT(8) * (t[c + sb] - t[c - sb]) - (t[c + 2 * sb] - t[c - 2 * sb])); };
            return R(8) * (u1(sa) - u1(-sa)) - (u1(2 * sa) - u1(-2 * sa));
        };
        // gradient and Hessian of the staged field
        auto grad_hess = [&](const P3& q, R* d, R* dd) {
            grad(q, d);
            dd[0] = (R(16) * q.x.a1 - q.x.a2) * fc.i12h2[0];
            dd[3] = (R(16) * q.y.a1 - q.y.a2) * fc.i12h2[1];
            dd[5] = (R(16) * q.z.a1 - q.z.a2) * fc.i12h2[2];
            dd[1] = mixd(1, SX) * fc.imix[0];
            dd[2] = mixd(1, SXY) * fc.imix[1];
            dd[4] = mixd(SX, SXY) * fc.imix[2];
        };

        // The right-hand side of each field is completed as soon as its inputs
        // exist, and every derivative block is folded into the terms it feeds
        // right after its field is staged, so that few values stay live across
        // the staging sequence (this decides how many waves a SIMD can hold).
        // Staging order: gt, Gt, W, alpha, Khat, Theta, beta, At, B.
        double k[NF];  // completed right-hand sides, stored by finish_point
        // --- conformal metric: first derivatives kept, second derivatives
        //     folded into -1/2 gt^lm d_l d_m gt_ij
        R Rt[6];
        R C2[3][6], Gtd[3];
        {
            R dgt[6][3];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                stage_field(q);
                const P3 pq = field_pairs();
                put_lds(P_AKGT + q, advko(pq));
                R dd[6];
                grad_hess(pq, dgt[q], dd);
                Rt[q] = R(-0.5) * tr6(gu, dd);
                pin(dgt[q]);
                pin(Rt[q]);
            }
            // Christoffel symbols: first kind C1[k][ij] = Gamma_kij, second kind C2[k][ij]
            R C1[3][6];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = i; j < 3; ++j)
                        C1[k][S(i, j)] = R(0.5) * (dgt[S(k, j)][i] + dgt[S(k, i)][j] - dgt[S(i, j)][k]);
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    C2[k][q] = gu[S(k, 0)] * C1[0][q] + gu[S(k, 1)] * C1[1][q] + gu[S(k, 2)] * C1[2][q];
#pragma unroll
            for (int k = 0; k < 3; ++k) Gtd[k] = tr6(gu, C2[k]);
            // gt^lm (2 Gamma^k_l(i Gamma_j)km + Gamma^k_im Gamma_klj) = M_ij + M_ji + T_ij with
            // Cu[a][b][l] = gt^lm Gamma_abm:  M_ij = C2[k][li] Cu[j][k][l],  T_ij = C2[k][im] Cu[k][j][m]
            R M[3][3], T3[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) M[i][j] = T3[i][j] = R(0);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    R cu[3];
#pragma unroll
                    for (int l = 0; l < 3; ++l)
                        cu[l] = gu[S(l, 0)] * C1[a][S(b, 0)] + gu[S(l, 1)] * C1[a][S(b, 1)] + gu[S(l, 2)] * C1[a][S(b, 2)];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        M[i][a] += C2[b][S(0, i)] * cu[0] + C2[b][S(1, i)] * cu[1] + C2[b][S(2, i)] * cu[2];
                        T3[i][b] += C2[a][S(i, 0)] * cu[0] + C2[a][S(i, 1)] * cu[1] + C2[a][S(i, 2)] * cu[2];
                    }
                }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = i; j < 3; ++j) {
                    R s = M[i][j] + M[j][i] + T3[i][j];
#pragma unroll
                    for (int k = 0; k < 3; ++k) s += R(0.5) * Gtd[k] * (C1[i][S(j, k)] + C1[j][S(i, k)]);
                    Rt[S(i, j)] += s;
                }
            pin(Rt);
            pin(C2);
            pin(Gtd);
        }

        // --- At at the point (its stencils are staged near the end): At^ij,
        //     At_ij At^ij and Gamma^a_jk At^jk now, so that C2 dies with the
        //     lapse below
        R At[6], Auu[6], AA, nG[3];  // nG: Gt source without advection/dissipation
        R mp[MON ? 3 : 1];           // monitor: M^i / W^2 without the gt gt d At term
        {
#pragma unroll
            for (int q = 0; q < 6; ++q) At[q] = get_lds(P_AT0 + q);
            R Au[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Au[i][j] = gu[S(i, 0)] * At[S(0, j)] + gu[S(i, 1)] * At[S(1, j)] + gu[S(i, 2)] * At[S(2, j)];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = i; j < 3; ++j)
                    Auu[S(i, j)] = Au[i][0] * gu[S(0, j)] + Au[i][1] * gu[S(1, j)] + Au[i][2] * gu[S(2, j)];
            AA = tr6(Auu, At);
#pragma unroll
            for (int a = 0; a < 3; ++a) nG[a] = tr6(C2[a], Auu);  // scaled by 2 alpha below
            if constexpr (MON) {
                // connection terms of the covariant divergence in M^i: with
                // Am_c^j = gt^jb At_cb,
                //   D_j At^ij = gt^ia gt^jb d_j At_ab - gt^ia Gamma^c_ja Am_c^j - Gtd^c Am_c^i
                // The monitor's products start from opaque copies (of At here):
                // a product it shared with the right-hand side (Am is At^i_j
                // there) would change how the compiler fuses multiplies and
                // adds in the right-hand side, and with them the stage's bits.
                const MonCopy<R, 6> a6(At);
                R Am[3][3];
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        Am[c][j] = gu[S(j, 0)] * a6.v[S(c, 0)] + gu[S(j, 1)] * a6.v[S(c, 1)] + gu[S(j, 2)] * a6.v[S(c, 2)];
                R Tm[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    R t = R(0);
#pragma unroll
                    for (int c = 0; c < 3; ++c)
#pragma unroll
                        for (int j = 0; j < 3; ++j) t += C2[c][S(j, a)] * Am[c][j];
                    Tm[a] = t;
                }
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    mp[i] = -(gu[S(i, 0)] * Tm[0] + gu[S(i, 1)] * Tm[1] + gu[S(i, 2)] * Tm[2])
                          - (Gtd[0] * Am[0][i] + Gtd[1] * Am[1][i] + Gtd[2] * Am[2][i]);
                pin(mp);
            }
            pin(At);
            pin(Auu);
            pin(AA);
            pin(nG);
        }

        // --- evolved Gt: Rt_ij += 1/2 (gt_ki d_j Gt^k + gt_kj d_i Gt^k)
        R Zu[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            stage_field(6 + a);
            const R Gam = tval(F_GAM + a);
            const P3 pq = field_pairs();
            put_lds(P_AKGAM + a, advko(pq));
            R d[3];
            grad(pq, d);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = i; j < 3; ++j) Rt[S(i, j)] += R(0.5) * (gt[S(a, i)] * d[j] + gt[S(a, j)] * d[i]);
            Zu[a] = R(0.5) * (Gam - Gtd[a]);
            pin(Rt);
            pin(Zu[a]);
        }

        // --- conformal factor: DDW_ij = d_i d_j W - Gamma^k_ij d_k W, folded
        //     into W^2 R_ij (no division by W)
        R W, dW[3], W2R[6], ak_w;
        {
            stage_field(9);
            W = tval(F_W);
            const P3 pq = field_pairs();
            ak_w = advko(pq);
            R DDW[6];
            grad_hess(pq, dW, DDW);
#pragma unroll
            for (int q = 0; q < 6; ++q) DDW[q] -= C2[0][q] * dW[0] + C2[1][q] * dW[1] + C2[2][q] * dW[2];
            const R trDDW = tr6(gu, DDW);
            R dW2 = R(0);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) dW2 += gu[S(i, j)] * dW[i] * dW[j];
#pragma unroll
            for (int q = 0; q < 6; ++q) W2R[q] = W * W * Rt[q] + W * (DDW[q] + gt[q] * trDDW) - R(2) * gt[q] * dW2;
            if constexpr (MON) {
                const MonCopy<R, 3> dw(dW);  // Auu . dW is also a term of the Gt source
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    mp[a] -= R(3) * (Auu[S(a, 0)] * dw.v[0] + Auu[S(a, 1)] * dw.v[1] + Auu[S(a, 2)] * dw.v[2]) / W;
                pin(mp);
            }
            pin(dW);
            pin(W2R);
        }
        // --- lapse: DDa_ij = d_i d_j alpha - Gamma^k_ij d_k alpha, folded into
        //     W^2 D_i D_j alpha and the trace-free source X_ij of At
        R al, ak_al, Ric, Lapa, Xtf[6];
        {
            stage_field(10);
            al = tval(F_AL);
            const P3 pq = field_pairs();
            ak_al = advko(pq);
            R da[3], DDa[6];
            grad_hess(pq, da, DDa);
#pragma unroll
            for (int q = 0; q < 6; ++q) DDa[q] -= C2[0][q] * da[0] + C2[1][q] * da[1] + C2[2][q] * da[2];
            R dWda = R(0);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) dWda += gu[S(i, j)] * dW[i] * da[j];
            R W2DDa[6];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = i; j < 3; ++j) {
                    const int q = S(i, j);
                    W2DDa[q] = W * W * DDa[q] + W * (dW[i] * da[j] + dW[j] * da[i] - gt[q] * dWda);
                }
            Ric = tr6(gu, W2R);
            Lapa = tr6(gu, W2DDa);
#pragma unroll
            for (int q = 0; q < 6; ++q) Xtf[q] = -W2DDa[q] + al * W2R[q];
            const R trX = tr6(gu, Xtf) * R(1.0 / 3.0);
#pragma unroll
            for (int q = 0; q < 6; ++q) Xtf[q] -= gt[q] * trX;
            const R iW = R(1) / (W > R(prm.w_floor) ? W : R(prm.w_floor));
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                R t_ada = R(0), t_aw = R(0);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    t_ada += Auu[S(a, c)] * da[c];
                    t_aw += Auu[S(a, c)] * dW[c];
                }
                nG[a] = R(-2) * t_ada + R(2) * al * nG[a] - R(6) * al * t_aw * iW;
            }
            pin(Xtf);
            pin(nG);
            pin(Ric);
            pin(Lapa);
        }
        // --- Khat and Theta: only the combination 2 d Khat + d Theta is used
        const R kap1 = R(prm.kappa1), kap3 = R(prm.kappa3);
        const R th1 = uniform(kap1 * (R(1) - R(prm.kappa2))), th2 = uniform(kap1 * (R(2) + R(prm.kappa2)));
        R K;
        double mon_h2 = 0.0;  // monitor: this wave's sum of H^2 (scalar registers)
        {
            stage_field(11);
            const R Kh = tval(F_KH);
            const P3 pk = field_pairs();
            const R ak_kh = advko(pk);
            R dkt[3];
            grad(pk, dkt);
            R dK[MON ? 3 : 1];  // monitor: d K = d Khat + 2 d Theta
            if constexpr (MON) {
#pragma unroll
                for (int j = 0; j < 3; ++j) dK[j] = dkt[j];
                pin(dK);
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) dkt[j] *= R(2);
            pin(dkt);
            stage_field(12);
            const R Th = tval(F_TH);
            const P3 pt = field_pairs();
            const R ak_th = advko(pt);
            R d[3];
            grad(pt, d);
#pragma unroll
            for (int j = 0; j < 3; ++j) dkt[j] += d[j];
            K = Kh + R(2) * Th;
            if constexpr (MON) {
                // -(2/3) gt^ij d_j K, and H = R - At_ij At^ij + (2/3) K^2.
                // The monitor forms its own d Theta from opaque copies of the
                // differences: a second use of the right-hand side's d Theta
                // products would keep the compiler from fusing them into the
                // sums 2 d Khat + d Theta, and change the stage's bits.
                const R tdif[6] = {pt.x.b1, pt.x.b2, pt.y.b1, pt.y.b2, pt.z.b1, pt.z.b2};
                const MonCopy<R, 6> db(tdif);
                const MonCopy<R, 6> g6(gu);
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    dK[j] += R(2) * ((R(8) * db.v[2 * j] - db.v[2 * j + 1]) * fc.i12h[j]);
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    mp[a] -= R(2.0 / 3.0) * (g6.v[S(a, 0)] * dK[0] + g6.v[S(a, 1)] * dK[1] + g6.v[S(a, 2)] * dK[2]);
                const MonCopy<R, 1> ric(&Ric), aa(&AA), kk(&K);
                const double H = double(ric.v[0] - aa.v[0] + R(2.0 / 3.0) * kk.v[0] * kk.v[0]);
                if (valid && mon.c) mon.c[p] = H;
                mon_h2 = wave_sum(valid ? H * H : 0.0);
                pin(mp);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const R t_dk = gu[S(a, 0)] * dkt[0] + gu[S(a, 1)] * dkt[1] + gu[S(a, 2)] * dkt[2];
                nG[a] -= R(2.0 / 3.0) * al * t_dk;
            }
            put_lds(P_KKH, -Lapa + al * (AA + K * K * R(1.0 / 3.0)) + al * th1 * Th + ak_kh);
            put_lds(P_KTH, R(0.5) * al * (Ric - AA + R(2.0 / 3.0) * K * K) - al * th2 * Th + ak_th);
            put_lds(P_KAL, R(-2) * al * (prm.lapse_uses_K ? K : Kh) + ak_al);
            pin(nG);
        }

        // --- shift: its first derivatives close the gt and At sources, the
        //     second derivatives the Gt source
        R kgt[6], kat[6];
        {
            R dbe[3][3], lapb[3], gdivb[3] = {R(0), R(0), R(0)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                stage_field(13 + a);
                const P3 pq = field_pairs();
                put_lds(P_AKBE + a, advko(pq));
                R dd[6];
                grad_hess(pq, dbe[a], dd);
                lapb[a] = tr6(gu, dd);
#pragma unroll
                for (int j = 0; j < 3; ++j) gdivb[j] += dd[S(j, a)];
                pin(dbe[a]);
                pin(lapb[a]);
                pin(gdivb);
            }
            const R divb = dbe[0][0] + dbe[1][1] + dbe[2][2];
            put_lds(P_KW, W * (al * K - divb) * R(1.0 / 3.0) + ak_w);
            R Au[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Au[i][j] = gu[S(i, 0)] * At[S(0, j)] + gu[S(i, 1)] * At[S(1, j)] + gu[S(i, 2)] * At[S(2, j)];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = i; j < 3; ++j) {
                    const int q = S(i, j);
                    R lg = R(0), la = R(0), aa = R(0);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        lg += gt[S(i, c)] * dbe[c][j] + gt[S(j, c)] * dbe[c][i];
                        la += At[S(i, c)] * dbe[c][j] + At[S(j, c)] * dbe[c][i];
                        aa += At[S(i, c)] * Au[c][j];
                    }
                    kgt[q] = R(-2) * al * At[q] + lg - R(2.0 / 3.0) * gt[q] * divb + get_lds(P_AKGT + q);
                    kat[q] = Xtf[q] + al * (K * At[q] - R(2) * aa) + la - R(2.0 / 3.0) * At[q] * divb;
                }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                R t_gdb = R(0), t_zdb = R(0), t_dd2 = R(0);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    t_gdb += Gtd[c] * dbe[a][c];
                    t_zdb += Zu[c] * dbe[a][c];
                    t_dd2 += gu[S(a, c)] * gdivb[c];
                }
                nG[a] += lapb[a] + t_dd2 * R(1.0 / 3.0) + R(2.0 / 3.0) * Gtd[a] * divb - t_gdb
                       - R(2) * al * kap1 * Zu[a] + R(2) * kap3 * (R(2.0 / 3.0) * Zu[a] * divb - t_zdb);
            }
            pin(kgt);
            pin(kat);
            pin(nG);
        }

        // --- traceless curvature and B: advection and dissipation only
        R mdiv[MON ? 3 : 1] = {};  // monitor: gt^ia gt^jb d_j At_ab
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            stage_field(16 + q);
            k[F_GT + q] = double(kgt[q]);
            const P3 pq = field_pairs();
            k[F_AT + q] = double(kat[q] + advko(pq));
            if constexpr (MON) {
                const MonCopy<R, 6> g6(gu);
                R d[3];
                grad(pq, d);
                pin(d);
                // component q = (c, e) stands for At_ce and At_ec
                const int c = q < 3 ? 0 : (q < 5 ? 1 : 2);
                const int e = q < 3 ? q : (q < 5 ? q - 2 : 2);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    R t = R(0);
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        R wgt = g6.v[S(a, c)] * g6.v[S(j, e)];
                        if (c != e) wgt += g6.v[S(a, e)] * g6.v[S(j, c)];
                        t += wgt * d[j];
                    }
                    mdiv[a] += t;
                }
                pin(mdiv);
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            stage_field(22 + a);
            const R Bc = tval(F_BB + a);
            const R ak_bb = advko(field_pairs());
            k[F_GAM + a] = double(nG[a] + get_lds(P_AKGAM + a));
            k[F_BE + a] = double(R(prm.shift_coeff) * Bc + get_lds(P_AKBE + a));
            k[F_BB + a] = double(nG[a] - R(prm.eta) * Bc + ak_bb);
        }
        k[F_KH] = double(get_lds(P_KKH));
        k[F_TH] = double(get_lds(P_KTH));
        k[F_AL] = double(get_lds(P_KAL));
        k[F_W] = double(get_lds(P_KW));

        if constexpr (MON) {
            double m2[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const MonCopy<R, 1> wm(&W);
                const double M = double(wm.v[0] * wm.v[0] * (mdiv[a] + mp[a]));
                if (valid && mon.c) mon.c[(size_t)(a + 1) * (size_t)B.sf + p] = M;
                m2[a] = wave_sum(valid ? M * M : 0.0);
            }
            if ((tid & 63) == 0) {
                double* a = mon_acc + (tid >> 6) * 4;
                a[0] += mon_h2;
                a[1] += m2[0];
                a[2] += m2[1];
                a[3] += m2[2];
            }
        }
        if (!valid) continue;  // no barrier below this point
        finish_point(B, mode, stage, [&](int f) { return k[f]; }, p);
    }
    if constexpr (MON) {
        // one record per wave of the grid, in brick order within the wave
        if ((tid & 63) == 0) {
            double* out = mon.part + ((size_t)blockIdx.x * (NT / 64) + (size_t)(tid >> 6)) * 4;
#pragma unroll
            for (int m = 0; m < 4; ++m) out[m] = mon_acc[(tid >> 6) * 4 + m];
        }
    }
}

// DMA staging moves 16-byte pairs: every tile row must start on an even
// element of a 16-byte aligned field (odd ghost width, even nx, even field
// stride, aligned base).
inline bool dma_compatible(const BoxSet& set)
{
    for (int b = 0; b < set.nbox; ++b) {
        const BoxDev& B = set.box[b];
        if (B.ng % 2 == 0 || B.n[0] % 2 != 0 || B.sf % 2 != 0 || ((uintptr_t)B.u_in & 15) != 0) return false;
    }
    return true;
}

template <typename R, int BX, int BY, int BZ, int WAVES, bool DMA, bool MON = false>
hipError_t launch_variant(const BoxSet& set, const ParamsDev& p, int mode, int stage, int persistent, hipStream_t s,
                          MonDev mon = MonDev{}, long* grid_out = nullptr)
{
    const long total = set.brick_begin[set.nbox];
    if (total <= 0) return hipSuccess;
    long grid = total;
    const BoxSet* run = &set;
    static int cap = 0;  // resident blocks per CU, x CUs; computed once per process
    if (cap == 0) {
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fused_stage<R, BX, BY, BZ, WAVES, DMA, MON>,
                                                           BX * BY * BZ, 0);
        cap = cus * (per > 0 ? per : 1);
    }
    if (persistent) {
        if (grid > cap) grid = cap;
    }
    grid = (grid + 7) / 8 * 8;  // whole XCD rounds (idle blocks exit at once)
    if (grid_out) *grid_out = grid;
    hipLaunchKernelGGL((fused_stage<R, BX, BY, BZ, WAVES, DMA, MON>), dim3((unsigned)grid), dim3(BX * BY * BZ), 0, s,
                       *run, p, mode, stage, mon);
    return hipGetLastError();
}

template <typename R, int BX, int BY, int BZ, int WAVES>
hipError_t launch_fused(const BoxSet& set, const ParamsDev& p, int mode, int stage, int persistent, hipStream_t s)
{
    if constexpr (BX % 2 == 0 && (BX * BY * BZ) % 64 == 0) {
        if (dma_compatible(set)) return launch_variant<R, BX, BY, BZ, WAVES, true>(set, p, mode, stage, persistent, s);
    }
    return launch_variant<R, BX, BY, BZ, WAVES, false>(set, p, mode, stage, persistent, s);
}

}  // namespace

// One float64 stage with the constraint monitor of its input (single box,
// 8x8x8 bricks with two waves per SIMD, persistent).  The launch leaves one
// record of four sums per wave of its grid (*records of them); the grid never
// exceeds the bricks rounded up to a multiple of 8.
long monitor_bricks(const int n[3]) { return (long)((n[0] + 7) / 8) * ((n[1] + 7) / 8) * ((n[2] + 7) / 8); }
long monitor_records_max(const int n[3]) { return (monitor_bricks(n) + 7) / 8 * 8 * 8; }
hipError_t launch_stage_monitor(const BoxSet& set, const ParamsDev& p, int mode, int stage, MonDev mon, hipStream_t s,
                                long* records)
{
    long grid = 0;
    hipError_t e = dma_compatible(set)
                       ? launch_variant<double, 8, 8, 8, 2, true, true>(set, p, mode, stage, 1, s, mon, &grid)
                       : launch_variant<double, 8, 8, 8, 2, false, true>(set, p, mode, stage, 1, s, mon, &grid);
    *records = grid * 8;
    return e;
}

namespace {

// ------------------------------------------------------------------------
// Ghost shells: thread q of a box enumerates its ghost points in the
// canonical order (k outermost, j, i fastest, active points skipped).
// ------------------------------------------------------------------------
__device__ __forceinline__ void shell_point(long q, int nx, int ny, int nz, int ng, int& i, int& j, int& k)
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

__device__ __forceinline__ int wrap(int i, int ng, int n)
{
    int a = (i - ng) % n;
    if (a < 0) a += n;
    return a + ng;
}

__device__ __forceinline__ int find_box(const BoxSet& set, long w)
{
    int bi = 0;
    while (w >= set.shell_begin[bi + 1]) ++bi;
    return bi;
}

// sign of field f under the reflection z -> -z: one factor -1 per z index
__device__ __forceinline__ double z_sign(int f)
{
    return (f == F_GT + 2 || f == F_GT + 4 || f == F_AT + 2 || f == F_AT + 4 || f == F_GAM + 2 || f == F_BE + 2 ||
            f == F_BB + 2)
               ? -1.0
               : 1.0;
}

// One thread per ghost point, all 25 fields.  Every load of a point is
// issued before its first store, so a thread keeps them all in flight (the
// stores may alias the sources as far as the compiler knows).
__global__ void __launch_bounds__(256) ghost_fill(BoxSet set)
{
    const long w = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= set.shell_begin[set.nbox]) return;
    const int bi = find_box(set, w);
    const BoxDev& B = set.box[bi];
    if (B.bc == Z4C_BC_SOMMERFELD) return;
    const long q = w - set.shell_begin[bi];
    const int Nx = B.n[0] + 2 * B.ng, Ny = B.n[1] + 2 * B.ng;
    // the shell order starts with the ng layers below the active box
    if (B.bc == Z4C_BC_EQUATORIAL && q >= (long)B.ng * Nx * Ny) return;
    int i, j, k;
    shell_point(q, B.n[0], B.n[1], B.n[2], B.ng, i, j, k);
    const size_t p = ((size_t)k * Ny + j) * Nx + i;
    double* u = const_cast<double*>(B.u_in);
    const size_t sf = (size_t)B.sf;
    double v[NF];
    if (B.bc == Z4C_BC_EQUATORIAL) {
        // layer ng-1-m below the symmetry plane mirrors layer ng+m above it
        const size_t src = ((size_t)(2 * B.ng - 1 - k) * Ny + j) * Nx + i;
#pragma unroll
        for (int f = 0; f < NF; ++f) v[f] = z_sign(f) * u[f * sf + src];
    } else if (B.bc == Z4C_BC_PERIODIC) {
        const size_t src = ((size_t)wrap(k, B.ng, B.n[2]) * Ny + wrap(j, B.ng, B.n[1])) * Nx + wrap(i, B.ng, B.n[0]);
#pragma unroll
        for (int f = 0; f < NF; ++f) v[f] = u[f * sf + src];
    } else {
        const size_t ns = (size_t)(set.shell_begin[bi + 1] - set.shell_begin[bi]);
        if (B.lv[2]) {
            // the shell at this stage time: weighted sum of the parent's time
            // levels, each prolonged in space (both steps are linear and commute)
#pragma unroll
            for (int f = 0; f < NF; ++f) v[f] = B.lw[1] * B.lv[1][f * ns + q] + B.lw[2] * B.lv[2][f * ns + q];
            if (B.lv[0]) {
#pragma unroll
                for (int f = 0; f < NF; ++f) v[f] += B.lw[0] * B.lv[0][f * ns + q];
            }
        } else {
            const double* sh = B.lv[1] ? B.lv[1] : B.shell;  // a stage time that is a time level
#pragma unroll
            for (int f = 0; f < NF; ++f) v[f] = sh[f * ns + q];
        }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) u[f * sf + p] = v[f];
    if (B.u_in2) {
#pragma unroll
        for (int f = 0; f < NF; ++f) B.u_in2[f * sf + p] = v[f];
    }
}

// 2nd-order derivative for the Sommerfeld condition: centred where both
// neighbours exist, one-sided inward at the array edge
__device__ __forceinline__ double dsomm(const double* u, size_t p, int i, int N, long st, double h)
{
    const double c = u[p];
    if (i >= 1 && i + 1 < N) return (u[p + st] - u[p - st]) / (2.0 * h);
    const long o = (i + 1 >= N) ? st : -st;  // upper edge leans on -1, -2
    const double s = (i + 1 >= N) ? 1.0 : -1.0;
    return s * (-4.0 * (u[p - o] - c) + (u[p - 2 * o] - c)) / (2.0 * h);
}

// Outgoing-wave update of the ghost points of Sommerfeld faces (every ghost
// of a Sommerfeld box; those at and above the symmetry plane of an
// equatorial box): d_t f = -(x^i/r) d_i f - (f - f_flat)/r (paper Sec.
// 2.2.2), then the same RK4 stage update and enforcement as the interior.
// Two threads per ghost point (blockIdx.y): one takes gt and At, whose
// enforcement needs all twelve, the other the 13 remaining fields, which
// doubles the loads in flight of this latency-bound update.
__global__ void __launch_bounds__(256) sommerfeld_ghosts(BoxSet set, int mode, int stage)
{
    const long w = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= set.shell_begin[set.nbox]) return;
    const int bi = find_box(set, w);
    const BoxDev& B = set.box[bi];
    if (B.bc != Z4C_BC_SOMMERFELD && B.bc != Z4C_BC_EQUATORIAL) return;
    const long q = w - set.shell_begin[bi];
    if (B.bc == Z4C_BC_EQUATORIAL && q < (long)B.ng * (B.n[0] + 2 * B.ng) * (B.n[1] + 2 * B.ng)) return;
    int i, j, k;
    shell_point(q, B.n[0], B.n[1], B.n[2], B.ng, i, j, k);
    const int Nx = B.n[0] + 2 * B.ng, Ny = B.n[1] + 2 * B.ng, Nz = B.n[2] + 2 * B.ng;
    const size_t p = ((size_t)k * Ny + j) * Nx + i;
    const size_t sf = (size_t)B.sf;
    const double x = B.x0[0] + (i - B.ng) * B.h[0];
    const double y = B.x0[1] + (j - B.ng) * B.h[1];
    const double z = B.x0[2] + (k - B.ng) * B.h[2];
    const double r = sqrt(x * x + y * y + z * z);
    const double ir = 1.0 / r;
    auto kf = [&](int f) {
        const double* u = B.u_in + f * sf;
        const double dr = (x * ir) * dsomm(u, p, i, Nx, 1, B.h[0]) + (y * ir) * dsomm(u, p, j, Ny, Nx, B.h[1])
                        + (z * ir) * dsomm(u, p, k, Nz, (long)Nx * Ny, B.h[2]);
        return -dr - (u[p] - flat_of(f)) * ir;
    };
    if (blockIdx.y == 0)
        finish_subset<true>(B, mode, stage, kf, p);
    else
        finish_subset<false>(B, mode, stage, kf, p);
}

__global__ void __launch_bounds__(256) zero_ghost_rhs(BoxSet set)
{
    const long w = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= set.shell_begin[set.nbox]) return;
    const int bi = find_box(set, w);
    const BoxDev& B = set.box[bi];
    if (B.bc == Z4C_BC_SOMMERFELD) return;
    const long q = w - set.shell_begin[bi];
    const int Nx = B.n[0] + 2 * B.ng, Ny = B.n[1] + 2 * B.ng;
    if (B.bc == Z4C_BC_EQUATORIAL && q >= (long)B.ng * Nx * Ny) return;  // Sommerfeld faces
    int i, j, k;
    shell_point(q, B.n[0], B.n[1], B.n[2], B.ng, i, j, k);
    const size_t p = ((size_t)k * Ny + j) * Nx + i;
#pragma unroll
    for (int f = 0; f < NF; ++f) B.u_out[f * (size_t)B.sf + p] = 0.0;
}

}  // namespace

hipError_t launch_ghosts(const BoxSet& set, hipStream_t s)
{
    const long total = set.shell_begin[set.nbox];
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(ghost_fill, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, set);
    return hipGetLastError();
}

hipError_t launch_sommerfeld(const BoxSet& set, const ParamsDev& p, int mode, int stage, hipStream_t s)
{
    (void)p;
    const long total = set.shell_begin[set.nbox];
    if (total <= 0) return hipSuccess;
    const dim3 grid((unsigned)((total + 255) / 256));
    hipLaunchKernelGGL(sommerfeld_ghosts, dim3(grid.x, 2), dim3(256), 0, s, set, mode, stage);
    if (mode == MODE_RHS) hipLaunchKernelGGL(zero_ghost_rhs, grid, dim3(256), 0, s, set);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Table of compiled tile shapes (first entry of each precision = default)
// ------------------------------------------------------------------------
template <typename R, int BX, int BY, int BZ, int WV>
hipError_t tile_resources(int* waves_per_simd, int* lds_bytes, int* scratch_bytes)
{
    const void* fn = reinterpret_cast<const void*>(&fused_stage<R, BX, BY, BZ, WV, true, false>);
    hipFuncAttributes fa{};
    hipError_t e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    int per = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fused_stage<R, BX, BY, BZ, WV, true, false>,
                                                          BX * BY * BZ, 0)) != hipSuccess)
        return e;
    *waves_per_simd = per * (BX * BY * BZ / 64) / 4;  // four SIMDs per compute unit
    *lds_bytes = (int)fa.sharedSizeBytes;
    *scratch_bytes = (int)fa.localSizeBytes;
    return hipSuccess;
}

#define Z4C_TILE(R, PREC, BX, BY, BZ, WV) \
    {{BX, BY, BZ, WV, 0}, PREC, &launch_fused<R, BX, BY, BZ, WV>, &tile_resources<R, BX, BY, BZ, WV>}

static const TileEntry kTiles[] = {
    Z4C_TILE(double, Z4C_FP64, 8, 8, 4, 1),
    Z4C_TILE(double, Z4C_FP64, 16, 4, 4, 1),
    Z4C_TILE(double, Z4C_FP64, 16, 8, 2, 1),
    Z4C_TILE(double, Z4C_FP64, 16, 2, 8, 1),
    Z4C_TILE(double, Z4C_FP64, 8, 4, 8, 1),
    Z4C_TILE(double, Z4C_FP64, 8, 8, 8, 2),
    Z4C_TILE(double, Z4C_FP64, 8, 8, 4, 2),
    Z4C_TILE(float, Z4C_MIXED, 8, 8, 4, 1),
    Z4C_TILE(float, Z4C_MIXED, 16, 4, 4, 1),
    Z4C_TILE(float, Z4C_MIXED, 8, 8, 4, 2),
    Z4C_TILE(float, Z4C_MIXED, 16, 8, 2, 2),
    Z4C_TILE(float, Z4C_MIXED, 8, 8, 8, 2),
};

int tile_table(const TileEntry** out)
{
    *out = kTiles;
    return (int)(sizeof(kTiles) / sizeof(kTiles[0]));
}

}  // namespace z4c
