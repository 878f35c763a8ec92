// Internal declarations shared by the HIP kernels and the C-ABI host code of
// libz4c.so.  Nothing here is part of the public interface (include/z4c.h).
#pragma once

#include <hip/hip_runtime.h>

#include "z4c.h"

namespace z4c {

constexpr int NF = 25;
constexpr int MAXBOX = 16;

// Field slots (same order as the public header).
enum Field : int {
    F_W = 0,
    F_GT = 1,   // gt_xx gt_xy gt_xz gt_yy gt_yz gt_zz
    F_KH = 7,
    F_AT = 8,   // At_xx .. At_zz
    F_GAM = 14, // Gt^x Gt^y Gt^z
    F_TH = 17,
    F_AL = 18,
    F_BE = 19,  // beta^x..z
    F_BB = 22   // B^x..z
};

// One box as the kernels see it.  Passed by value inside BoxSet.
struct BoxDev {
    const double* u_in;   // stage input (stencil reads; ghosts valid)
    const double* u_n;    // state at the start of the step (stages 2, 3)
    double* acc;          // RK4 accumulator
    double* u_out;        // stage output, or the right-hand side in RHS mode
    const double* shell;  // ghost shell (copy boxes)
    // Copy boxes of a patch hierarchy instead read the parent's time levels
    // prolonged in space and fill each ghost with their weighted sum
    // lw[1] lv[1] + lw[2] lv[2] (+ lw[0] lv[0] where lv[0] is set); with
    // lv[2] NULL, lv[1] alone is the shell (a stage time that is a level).
    const double* lv[3];
    double lw[3];
    double* u_in2;        // ghost fill only: a second array that takes the same ghosts (NULL: none)
    long sf;              // stride between fields
    int n[3];             // active cells
    int ng;               // ghost width
    int bc;               // z4c_bc
    int nb[3];            // bricks per direction (fused kernel)
    double h[3];
    double x0[3];
    double dt;
};

// Several boxes in one launch.  brick_begin / shell_begin are exclusive
// prefix sums of the per-box work counts of the fused and the ghost kernels.
struct BoxSet {
    int nbox;
    long brick_begin[MAXBOX + 1];
    long shell_begin[MAXBOX + 1];
    BoxDev box[MAXBOX];
};
static_assert(sizeof(BoxSet) + 256 <= 4096, "a BoxSet and the scalars beside it must fit the kernel arguments");

struct ParamsDev {
    double kappa1, kappa2, kappa3, eta, shift_coeff, ko_sigma, w_floor;
    int lapse_uses_K;
};

// mode of the fused kernel
enum Mode : int { MODE_RHS = 0, MODE_STAGE = 1 };

// Outputs of the constraint monitor fused into a stage (unused otherwise).
struct MonDev {
    double* c;     // NULL or 4 fields of the box's stride: H, M^x, M^y, M^z at the active points
    double* part;  // per wave of the grid: sums of H^2, (M^x)^2, (M^y)^2, (M^z)^2 over its bricks
};
// a float64 stage (or RHS) of one box with the monitor of its input; bricks
// of 8^3, eight waves each.  part takes at most monitor_records_max(n) * 4
// doubles; *records is the number the launch writes.
long monitor_bricks(const int n[3]);
long monitor_records_max(const int n[3]);
hipError_t launch_stage_monitor(const BoxSet& set, const ParamsDev& p, int mode, int stage, MonDev mon, hipStream_t s,
                                long* records);
// fixed-order sum of n partial rows of 4 and the four L2 norms sqrt(sum / cells)
hipError_t launch_norms(const double* partial, long n, double inv_cells, double* norms, hipStream_t s);
hipError_t launch_zero(double* x, long n, hipStream_t s);

// Compiled tile shapes.
struct TileEntry {
    z4c_tile tile;
    int precision;
    // enqueue the fused kernel over every brick of `set`
    hipError_t (*launch)(const BoxSet& set, const ParamsDev& p, int mode, int stage, int persistent,
                         hipStream_t s);
    // resources of the shape's LDS-DMA kernel (the one aligned boxes run):
    // resident waves per SIMD, static LDS bytes per block, scratch bytes per lane
    hipError_t (*resources)(int* waves_per_simd, int* lds_bytes, int* scratch_bytes);
};

int tile_table(const TileEntry** out);  // returns the number of entries

hipError_t launch_ghosts(const BoxSet& set, hipStream_t s);                  // periodic / copy fill
hipError_t launch_sommerfeld(const BoxSet& set, const ParamsDev& p, int mode, int stage, hipStream_t s);

// constraint monitor (single box): per-point values (c may be NULL), block
// partial sums of C^2 into ws, then the four L2 norms into norms
long constraint_blocks(const int n[3]);
hipError_t launch_constraints(const BoxSet& set, double* c_out, double* norms, double* ws, hipStream_t s);

// ---------------------------------------------------------------------------
// Device helpers shared by the stencil kernels (LDS tile staging).
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void;

// s_waitcnt immediates (gfx9 encoding): vmcnt <= n with the other counters
// unconstrained, and lgkmcnt = 0
#define VM_N(n) ((((n) & 0xF) | ((((n) >> 4) & 0x3) << 14)) | (0x7 << 4) | (0xF << 8))
#define LGKM0 (0xF | (0x3 << 14) | (0x7 << 4))

// One LDS-DMA load: every lane moves the 16 bytes at `src` to LDS address
// `dst` + 16 * lane (dst uniform).  Issued as inline assembly so that the
// compiler's wait-count insertion does not see it: it would otherwise treat
// every outstanding tile load as a pending write to any LDS address and drain
// all of them (vmcnt(0)) before the next LDS read, which defeats loading
// tiles ahead of their use.  The kernels wait for these loads themselves
// (per-field vmcnt waits and a barrier before a tile is read); the loads
// complete in issue order with the compiler's own loads, so its waits for
// those stay correct (they may only wait longer).
__device__ __forceinline__ void lds_dma16(const void* src, lds_void* dst)
{
    const unsigned m = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long)dst);
    __asm__ volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                     :
                     : "v"(src), "s"(m)
                     : "memory", "m0");
}

// Workgroup barrier without a memory fence (s_barrier alone): the caller
// waits for exactly the LDS writes it needs with s_waitcnt, so that later
// tiles' loads stay in flight across it.  The empty asm statements keep the
// compiler from moving memory accesses across the barrier.
__device__ __forceinline__ void bar()
{
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
}

// Inter-level transfers of the Berger-Oliger hierarchy.
// One patch of a hierarchy depth as the transfer kernels see it.  Lattice
// index G of a cell at the patch's depth: active cell a of the patch sits at
// G = off + a (all patches of one depth share the lattice).
constexpr int MAXEX = 16;  // patches of one depth a transfer launch can take
struct PatchRef {
    double* u;
    long sf;
    int N[3];    // stored extents
    int n[3];    // active extents
    int ng;
    int off[3];
};
// Spatial prolongation of one parent level into a child's ghost shell,
// evaluated in three separable passes through scratch (6-point sums nearest
// node first, x innermost, then y, then z): X holds the x sums for every child x
// index and every parent (y, z) row used, Y the y sums for every child
// (x, y) and parent z row, the last pass the z sums at the shell points.
struct SepArgs {
    const double* u;  // parent level
    long sfp;
    int Np[3];        // parent stored extents
    int ngp;
    int nc[3];        // child active extents
    int ngc;
    int F[3];
    int Y0, NY;       // parent active y rows Y0 .. Y0+NY-1 held in X
    int Z0, NZ;       // parent active z rows Z0 .. Z0+NZ-1 held in X and Y
    double* X;        // 25 x NZ x NY x (nc[0]+2ngc)
    double* Y;        // 25 x NZ x (nc[1]+2ngc) x (nc[0]+2ngc)
    double* shell;
    long nshell;
    int refl;         // the child's lower z face is a symmetry plane: parent rows below it are mirror images
    // Parent rows (active index, after reflection) that the child's lower and
    // upper ghost layers read in z (zf) and in y (yf), as two intervals
    // {lo0, hi0, lo1, hi1}.  Columns of the child's active x-y interior need
    // y sums only in the zf rows, and those need x sums only in the yf rows;
    // the passes skip every other entry of an interior column or row.
    int zf[4];
    int yf[4];
};
struct RestrictArgs {
    PatchRef child[MAXEX];  // every patch of the finer depth (active cells and one ghost layer read)
    int nchild;
    PatchRef parent;        // covered active cells overwritten
    int lo[3], ext[3];      // parent active cells handled (parent active index)
};
struct ExchArgs {
    PatchRef p[MAXEX];  // every patch of the depth, in index order
    int np;
    int t;              // the patch this launch works for
    int lo[3], ext[3];  // lattice cells handled
};
struct ShiftArgs {
    const double* uc;  // the patch before the shift
    double* out;       // the patch after it (active cells written)
    long sfc;
    int Nc[3];
    int ngc;
    int nc[3];
    int s[3];          // shift in parent cells (2 s own cells), each -1, 0 or 1
    const double* up;  // parent state (same time)
    long sfp;
    int Np[3];
    int ngp;
    int F[3];          // parent active cell index of the shifted patch's lower faces
    int refl;          // the patch lies on the symmetry plane: parent rows below it are mirror images
};
struct TrackArgs {
    double* state;  // device: x[3], b0[3], xs[3], error flag
    const double* u;  // level whose shift is interpolated
    long sf;
    int N[3];
    int ng;
    double x0[3], h[3];
    double dt;
    int mode;  // 0: predictor (before the step), 1: corrector (after it)
    int refl;  // the level's lower z face is a symmetry plane: layers below it are mirror images
};
// Several prolongations in one launch per pass (each with its own part of
// the scratch); b* are exclusive prefix sums of the passes' thread counts,
// each rounded up to whole 256-thread blocks (batch_add).
constexpr int MAXSEP = 16;
struct SepBatch {
    int n;
    long bx[MAXSEP + 1], by[MAXSEP + 1], bz[MAXSEP + 1];
    SepArgs e[MAXSEP];
};
static_assert(sizeof(SepBatch) + 256 <= 4096, "a SepBatch must fit the kernel arguments");
// threads of the three passes of one prolongation, per field (the x and y
// sums of all 25 fields take 25 times nx and ny doubles of scratch)
void sep_counts(const SepArgs& a, long& nx, long& ny, long& nz);
// next exclusive prefix sum: an entry of `count` threads starts a block
inline long batch_add(long begin, long count) { return begin + (count + 255) / 256 * 256; }
hipError_t launch_prolong_sep(const SepBatch& b, hipStream_t s);
hipError_t launch_shift(const ShiftArgs& a, hipStream_t s);
// the puncture updates of several objects, one block each
struct TrackBatch {
    int n;
    TrackArgs a[MAXEX];
};
static_assert(sizeof(TrackBatch) + 256 <= 4096, "a TrackBatch must fit the kernel arguments");
hipError_t launch_track(const TrackBatch& b, hipStream_t s);
hipError_t launch_restrict(const RestrictArgs& a, hipStream_t s);
hipError_t launch_exchange_average(const ExchArgs& a, hipStream_t s);
hipError_t launch_exchange_ghosts(const ExchArgs& a, hipStream_t s);
// Copy of the stored-coordinate box [lo, lo + ext) of all 25 fields
// between two arrays of one patch's layout (stored extents N, field stride sf).
struct CopyBoxArgs {
    double* dst;
    const double* src;
    long sf;
    int N[3];
    int lo[3];
    int ext[3];
};
struct CopyBoxBatch {
    int n;
    long begin[MAXEX + 1];  // exclusive prefix sums of 25 x box cells (batch_add)
    CopyBoxArgs e[MAXEX];
};
static_assert(sizeof(CopyBoxBatch) + 256 <= 4096, "a CopyBoxBatch must fit the kernel arguments");
hipError_t launch_copy_box(const CopyBoxBatch& b, hipStream_t s);
// several flat copies of n[i] doubles in one launch
struct CopyList {
    int n;
    long begin[MAXEX + 1];  // batch_add of len
    long len[MAXEX];
    double* dst[MAXEX];
    const double* src[MAXEX];
};
hipError_t launch_copy_list(const CopyList& c, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, long n, hipStream_t s);
// out = w0 s0 + w1 s1 + w2 s2 over n doubles (s0 may be NULL)

}  // namespace z4c
