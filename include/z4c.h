/*
 * z4c.h -- C ABI of the MI355X (gfx950) Z4c evolution library, libz4c.so.
 *
 * What the library computes (paper: "SACRA-K", arXiv 2607.08743):
 *   - the right-hand side of the 25 evolved spacetime fields of Sec. 2.1.1
 *     (W, gt_ij, Khat, At_ij, Gt^i, Theta, alpha, beta^i, B^i) in the W form
 *     of the Z4c system the paper adopts (Sec. 2.1.1), with 1+log slicing and
 *     the Gamma-driver shift (Sec. 2.1.1, gauge equations);
 *   - 4th-order centred and shift-upwinded differences and 6th-order
 *     Kreiss-Oliger dissipation (Sec. 2.2, spatial discretisation);
 *   - the classical RK4 substep of the method of lines (Sec. 2.2), fused with
 *     the right-hand side and with the restoration of det gt = 1 and
 *     tr At = 0 (stated in Sec. 2.1.1);
 *   - outer-boundary treatment: periodic wrap, copy from a fixed ghost shell,
 *     or the Sommerfeld outgoing condition of Sec. 2.2.2;
 *   - a batched form that advances every box of a box-in-box hierarchy
 *     (Sec. 2.2.1) with one launch per substep, replayed as a HIP graph.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array pointer is a DEVICE pointer owned by the caller (the
 * library never frees it).  State arrays are float64, structure of arrays,
 * field-major with x fastest:
 *     u[f*sf + (k*Ny + j)*Nx + i],  Nx = nx + 2 ng, Ny = ny + 2 ng, Nz = nz + 2 ng,
 *     0 <= f < 25, 0 <= i < Nx (likewise j, k),  sf >= Nx*Ny*Nz (padding allowed).
 * Field order: 0 W | 1..6 gt_xx gt_xy gt_xz gt_yy gt_yz gt_zz | 7 Khat |
 * 8..13 At_xx..At_zz | 14..16 Gt^x..z | 17 Theta | 18 alpha | 19..21 beta^x..z |
 * 22..24 B^x..z.
 * Grid.  Cell-centred (Sec. 2.2.1): active cells are i in [ng, ng+nx); the
 * centre of stored point i is x0 + (i - ng)*dx, so x0 is the centre of the
 * first active cell.  ng >= 3 (the stencils reach 3 cells).
 * Streams.  `stream` is a hipStream_t (NULL = default stream).  Calls only
 * enqueue work and return; a fault inside a kernel surfaces at the caller's
 * next synchronisation or as Z4C_EHIP from a later call.
 * Errors.  Arguments are validated on the host before anything is enqueued;
 * an invalid call returns a negative z4c_status, enqueues nothing and leaves
 * a description in z4c_last_error().  Only the plan, tuning and hierarchy
 * APIs allocate (at creation, z4c_autotune's temporary plan, and
 * z4c_hier_set_moving).  No entry point synchronises the device except the
 * autotuners while they time (z4c_autotune on a cache miss,
 * z4c_plan_autotune) and the hierarchy's puncture read-back
 * (z4c_hier_advance with moving patches, z4c_hier_puncture).
 * Threads.  The single-box entry points are stateless and thread safe; a
 * plan or a hierarchy must not be used from two threads at once.
 */
#ifndef Z4C_H
#define Z4C_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    Z4C_OK = 0,
    Z4C_EINVAL = -1,       /* invalid argument (nothing enqueued) */
    Z4C_EHIP = -2,         /* the HIP runtime reported an error */
    Z4C_ENOMEM = -3,       /* device or host allocation failed (plan and hierarchy APIs only) */
    Z4C_EUNSUPPORTED = -4  /* valid request the compiled library cannot serve (e.g. no such tile) */
} z4c_status;

typedef enum {
    Z4C_BC_PERIODIC = 0,   /* ghosts wrap around the active box */
    Z4C_BC_SOMMERFELD = 1, /* ghost points are evolved with the outgoing-wave condition (Sec. 2.2.2) */
    Z4C_BC_COPY = 2,       /* ghosts are copied from a caller-owned shell (stand-in for AMR/neighbour data) */
    Z4C_BC_EQUATORIAL = 3  /* equatorial symmetry (Sec. 2.4, the paper's octant/equatorial runs): the lower z
                              face of the active box is the plane z = 0; ghost layer ng-1-m is layer ng+m
                              times (-1)^(number of z indices of the component), filled by apply_ghosts;
                              the other five faces are Sommerfeld faces whose ghosts are evolved.  Place
                              the box at z0 = dz/2 for the outgoing-wave terms to see z >= 0. */
} z4c_bc;

typedef enum {
    Z4C_FP64 = 0,  /* all arithmetic in float64 */
    Z4C_MIXED = 1  /* stencil and right-hand-side arithmetic in float32; state, RK4 accumulation and
                      constraint enforcement in float64 */
} z4c_precision;

/* Physical and numerical parameters.
 *   kappa1, kappa2   Z4c constraint damping (paper runs: 0.005, 0; Sec. 3)
 *   kappa3           factor of the non-principal Z terms of the Gt equation (0 = off)
 *   eta              Gamma-driver damping (paper runs: 0.36; Sec. 3)
 *   shift_coeff      Gamma-driver coefficient (0.75; Sec. 2.1.1)
 *   ko_sigma         Kreiss-Oliger coefficient (0.5; Sec. 2.2)
 *   w_floor          lower bound on W where 1/W appears (1e-10)
 *   lapse_uses_K     0: 1+log uses Khat (default); 1: it uses Khat + 2 Theta
 *   precision        z4c_precision */
typedef struct z4c_params {
    double kappa1, kappa2, kappa3, eta, shift_coeff, ko_sigma, w_floor;
    int lapse_uses_K;
    int precision;
} z4c_params;

/* Fill *p with the defaults listed above (FP64).  Never fails for p != NULL. */
void z4c_default_params(z4c_params* p);

/* Right-hand side of the 25 fields (Sec. 2.1.1 equations, Sec. 2.2 stencils).
 * Writes rhs on every active point; on a Z4C_BC_SOMMERFELD box also on every
 * ghost point, on a Z4C_BC_EQUATORIAL box on the ghost points at and above
 * the symmetry plane (the outgoing-wave right-hand side of Sec. 2.2.2); every
 * other ghost entry of rhs is set to 0.  Precondition: the ghosts of u are valid
 * (apply_ghosts for periodic/copy boxes).  u and rhs must not overlap.
 * Uses the default tile.  Returns Z4C_OK or an error as above. */
int rhs_z4c(const double* u, double* rhs, long sf, int nx, int ny, int nz, int ng, double dx, double dy,
            double dz, double x0, double y0, double z0, int bc, const z4c_params* p, void* stream);

/* One fused classical-RK4 substep (Sec. 2.2): k = RHS(u_in), then
 *   stage 1:  u_out = E(u_in + dt/2 k),  acc  = u_in + dt/6 k     (u_n is not read; may be NULL)
 *   stage 2:  u_out = E(u_n  + dt/2 k),  acc += dt/3 k
 *   stage 3:  u_out = E(u_n  + dt   k),  acc += dt/3 k
 *   stage 4:  u_out = E(acc  + dt/6 k)                              (u_n is not read; may be NULL)
 * where E restores det gt = 1 and tr At = 0 (gt <- gt/cbrt(det gt), then
 * At <- At - gt (gt^kl At_kl)/3), always in float64.  Points written: the
 * active points, plus the ghost points of Sommerfeld faces (every ghost of a
 * Sommerfeld box, those at and above the plane of an equatorial box); the
 * other ghosts are left for apply_ghosts.  Preconditions: ghosts of u_in valid.
 * Aliasing: u_out must differ from u_in and acc; acc must differ from u_in
 * and u_n; u_out == u_n is allowed only in stage 4 (the usual rotation is
 * u_n -> A -> B -> A -> u_n).  dt > 0, 1 <= stage <= 4. */
int rk4_substep(int stage, double dt, const double* u_in, const double* u_n, double* acc, double* u_out, long sf,
                int nx, int ny, int nz, int ng, double dx, double dy, double dz, double x0, double y0, double z0,
                int bc, const z4c_params* p, void* stream);

/* rk4_substep fused with the constraint monitor of its input (Sec. 2.3):
 * the same stage (bitwise the same u_out and acc), and from the same staged
 * fields and derivatives the Hamiltonian and momentum constraints of u_in
 * (definitions as for z4c_constraints) at every active point, plus their
 * volume-normalised L2 norms.  Stage 1 of an RK4 step thus monitors the state
 * at the start of the step at a small fraction of a separate monitor's cost.
 * Float64 only (Z4C_EUNSUPPORTED otherwise); always 8x8x8 bricks with two
 * waves per SIMD, persistent.
 *   c      device, NULL or 4 fields of stride sf (H, M^x, M^y, M^z); ghost entries set to 0
 *   norms  device, 4 doubles
 *   ws     device workspace of ws_len >= z4c_monitor_workspace(nx, ny, nz) doubles
 *          (an upper bound; one record of four sums per wave of the launch,
 *          each wave summing its bricks in the order it walks them, and the
 *          norms sum the records in a fixed order: bitwise reproducible run
 *          to run on one device, though not bitwise those of z4c_constraints,
 *          whose reduction tree differs)
 * c, norms and ws must not overlap each other or the state arrays.  Other
 * arguments, aliasing rules and errors as for rk4_substep. */
long z4c_monitor_workspace(int nx, int ny, int nz);
int rk4_substep_monitor(int stage, double dt, const double* u_in, const double* u_n, double* acc, double* u_out,
                        long sf, int nx, int ny, int nz, int ng, double dx, double dy, double dz, double x0, double y0,
                        double z0, int bc, const z4c_params* p, double* c, double* norms, double* ws, long ws_len,
                        void* stream);

/* Fill the ghost points of u (in place).  Z4C_BC_PERIODIC: wrap from the
 * active box.  Z4C_BC_COPY: copy from `shell`, a float64 array of shape
 * (25, nshell), nshell = Nx*Ny*Nz - nx*ny*nz, holding the ghost points in
 * the order (k outermost, then j, then i fastest) with active points skipped.
 * Z4C_BC_EQUATORIAL: the ng layers below the symmetry plane, every i and j,
 * from their mirror layers with the z parity of each field (the other ghosts
 * are evolved and must be valid already).
 * Z4C_BC_SOMMERFELD: nothing to do (the ghosts are evolved); returns Z4C_OK.
 * `shell` must be NULL unless bc == Z4C_BC_COPY. */
int apply_ghosts(double* u, const double* shell, long sf, int nx, int ny, int nz, int ng, int bc, void* stream);

/* Constraint monitor (Sec. 2.3): the Hamiltonian constraint
 *   H = R - At_ij At^ij + (2/3) K^2              (K = Khat + 2 Theta)
 * and the momentum constraint
 *   M^i = W^2 [ Dt_j At^ij - 3 At^ij d_j W / W - (2/3) gt^ij d_j K ]
 * of the vacuum 3+1 equations, on every active point, with R assembled as in
 * the right-hand side (evolved Gt in its d Gt term) and the 4th-order
 * centred stencils of Sec. 2.2; and their volume-normalised L2 norms
 * sqrt(sum C^2 / ncells) over the active cells (uniform cells: the dV
 * weights cancel).  Precondition: ghosts of u valid.
 *   c        device, NULL or 4 fields of stride sf (H, M^x, M^y, M^z); ghost
 *            entries are set to 0.  Must not overlap u.
 *   norms    device, 4 doubles (same order).
 *   ws       device workspace of ws_len >= z4c_constraints_workspace(nx, ny,
 *            nz) doubles, caller-owned, overwritten.
 * The reduction order is fixed by the box size, so the norms are bitwise
 * reproducible.  Nothing is allocated. */
long z4c_constraints_workspace(int nx, int ny, int nz);
int z4c_constraints(const double* u, double* c, double* norms, double* ws, long ws_len, long sf, int nx, int ny,
                    int nz, int ng, double dx, double dy, double dz, void* stream);

/* z4c_constraints for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same kernels and the same fixed-order
 * reduction, with the block partial sums kept in a fixed device array of the
 * library (16 MiB, one copy per device, held until the process ends).  Hence
 * at most Z4C_CONSTRAINTS_NOALLOC_MAX_BLOCKS bricks of 8x8x4 active cells
 * (a 512^3 box); a larger box fails with Z4C_EINVAL and enqueues nothing.
 * Results are bitwise those of z4c_constraints.  Calls no hipMalloc or
 * hipFree; the first call on a device looks the array's address up.  Every
 * call on one device shares that array: calls that overlap on a device
 * (other streams, other threads) race and must be serialised by the caller. */
#define Z4C_CONSTRAINTS_NOALLOC_MAX_BLOCKS 524288
int z4c_constraints_noalloc(const double* u, double* c, double* norms, long sf, int nx, int ny, int nz, int ng,
                            double dx, double dy, double dz, void* stream);

/* ---------------------------------------------------------------------- */
/* Batched form: every box of a hierarchy (Sec. 2.2.1 box-in-box levels)  */
/* in one persistent launch per substep, captured once as a HIP graph.    */
/* ---------------------------------------------------------------------- */

/* One box of a plan.  u_n holds the state and is advanced in place;
 * u_a, u_b (stage states) and acc are caller-owned scratch arrays of the
 * same shape.  dt is this box's own step (no subcycling).  shell: COPY
 * boxes only (see apply_ghosts), else NULL. */
typedef struct z4c_box {
    int n[3];
    int ng;
    int bc;
    long sf;
    double dx[3];
    double x0[3];
    double dt;
    double* u_n;
    double* u_a;
    double* u_b;
    double* acc;
    const double* shell;
} z4c_box;

/* Tile shape of the fused kernel: a brick of bx*by*bz points (one point per
 * thread) staged through LDS with a 3-cell halo; `waves` is the minimum
 * number of resident waves per SIMD the kernel is compiled for; `persistent`
 * caps the grid at (CUs * resident blocks) and loops over bricks.  The set of
 * compiled shapes is fixed; z4c_tile_count/z4c_tile_get enumerate it. */
typedef struct z4c_tile {
    int bx, by, bz, waves, persistent;
} z4c_tile;

int z4c_tile_count(int precision);
int z4c_tile_get(int precision, int index, z4c_tile* out);

/* Choose the tile shape (and persistent flag) that rhs_z4c and rk4_substep
 * use for `precision` (process-wide, thread safe); tile == NULL restores the
 * default (8x8x8 bricks with two waves per SIMD where compiled, else the
 * first shape; not persistent).  Z4C_EUNSUPPORTED if that shape is not
 * compiled. */
int z4c_select_tile(int precision, const z4c_tile* tile);

/* Resources of the compiled kernel of one tile shape (the LDS-DMA form that
 * boxes with 16-byte aligned rows run; tile->persistent is ignored), as the
 * HIP runtime reports them for the current device: resident waves per SIMD
 * (occupancy), static LDS bytes per block, scratch (register spill) bytes per
 * lane.  Outputs are host ints.  Z4C_EINVAL for an unknown precision or a
 * NULL argument, Z4C_EUNSUPPORTED if the shape is not compiled, Z4C_EHIP if
 * the runtime query fails.  Enqueues nothing. */
int z4c_tile_resources(int precision, const z4c_tile* tile, int* waves_per_simd, int* lds_bytes,
                       int* scratch_bytes);

/* Where a plan's tile shape came from (z4c_plan_tile, z4c_autotune). */
typedef enum {
    Z4C_TILE_DEFAULT = 0, /* the library default (8x8x8 bricks, two waves per SIMD, persistent) */
    Z4C_TILE_CALLER = 1,  /* the tile argument of z4c_plan_create */
    Z4C_TILE_CACHE = 2,   /* an entry of the tuning cache */
    Z4C_TILE_TUNED = 3    /* timed by z4c_autotune / z4c_plan_autotune in this process */
} z4c_tile_source;

/* Create a plan over nbox boxes (1 <= nbox <= 16, largest first is best).
 * The tile shape: `tile` if not NULL; else the entry of the tuning cache
 * `tune_cache_path` (see z4c_autotune) for this device, precision, box count
 * and workload bucket, if there is one and its shape is compiled; else the
 * library default shape for p->precision with a persistent launch.  A
 * missing cache file is an empty cache; an unreadable or corrupt one fails
 * with Z4C_EINVAL.  Allocates only host memory; queries the current device's
 * architecture when the cache holds entries.  *plan receives an opaque
 * handle. */
int z4c_plan_create(const z4c_box* boxes, int nbox, const z4c_params* p, const z4c_tile* tile,
                    const char* tune_cache_path, void** plan);

/* The tile shape (with its persistent flag) a plan launches and where it came
 * from (z4c_tile_source); either output may be NULL. */
int z4c_plan_tile(void* plan, z4c_tile* tile, int* source);

/* Advance every box by nsteps RK4 steps on `stream`: per step, four
 * substeps, each one ghost-fill launch and one fused launch over all
 * boxes.  The first call captures one step as a HIP graph; every call
 * replays it nsteps times (use_graph = 0 launches the kernels directly). */
int z4c_plan_step(void* plan, int nsteps, int use_graph, void* stream);

/* Time one RK4 step of the plan for every compiled tile shape, each with
 * persistent = 0 and 1 (median of `reps` after one warm-up step, HIP events
 * on `stream`), keep the fastest in the plan and write it to *best (if not
 * NULL).  The boxes' state is advanced by the trial steps, so callers reset
 * it afterwards.  ms (if not NULL) must hold 2*z4c_tile_count(precision)
 * floats: ms[2*i + persistent] receives the time of shape i. */
int z4c_plan_autotune(void* plan, int reps, void* stream, z4c_tile* best, float* ms);

int z4c_plan_destroy(void* plan);

/* The project's autotuner with a persisted cache (box-in-box batching of
 * Sec. 2.2.1 run as one launch per substep; the tile is the LDS brick of the
 * stencil staging).  Looks up (device architecture, p->precision, nbox,
 * bucket = floor(log2(total active cells))) in tune_cache_path; on a hit
 * returns the cached shape without running anything (*source =
 * Z4C_TILE_CACHE).  On a miss it builds a temporary plan over the boxes, times
 * one RK4 step for every compiled shape, persistent and not (median of 2
 * after a warm-up step, HIP events on `stream`), writes the fastest to the
 * cache (replacing the key's entry, file rewritten through a temporary file
 * and a rename) and returns it (*source = Z4C_TILE_TUNED).  The trial steps
 * advance the boxes' state: callers reset it afterwards.  tune_cache_path ==
 * NULL times without persisting.  The cache is a text file of JSON lines,
 *   {"arch": "gfx950", "precision": 0, "nbox": 1, "bucket": 24, "tile": [8, 8, 8, 2, 1], "ms": 29.4}
 * one per key; a line that is not such an entry makes the file corrupt
 * (Z4C_EINVAL, nothing timed, the file left as it is).  best and source may be
 * NULL.  Synchronises on `stream` when it times. */
int z4c_autotune(const z4c_box* boxes, int nbox, const z4c_params* p, const char* tune_cache_path, void* stream,
                 z4c_tile* best, int* source);

/* Host-only cache query: the cached shape for architecture `arch` (e.g.
 * "gfx950"), precision, and the box count and bucket of `boxes` (only their
 * extents n are read).  Returns 1 and fills *tile on a hit, 0 on a miss (also
 * for a missing file or a shape the library does not compile), Z4C_EINVAL for
 * a corrupt file or invalid arguments.  Makes no HIP call. */
int z4c_tune_lookup(const char* tune_cache_path, const char* arch, const z4c_box* boxes, int nbox, int precision,
                    z4c_tile* tile);

/* ---------------------------------------------------------------------- */
/* Box-in-box hierarchy with Berger-Oliger time subcycling (Sec. 2.2.1,   */
/* Fig. 1): a list of patches; patch 0 is the root (the coarsest level,   */
/* with its own boundary), every other patch names its parent, which it   */
/* refines 2:1.  A patch at depth d advances with dt0 / 2^d, two steps    */
/* per parent step, together with every patch of its depth (one launch    */
/* per RK4 stage).  Fixed levels are single patches; a moving level holds */
/* one patch per tracked object.  A patch's ghost zone comes from its     */
/* parent by 6th-order Lagrange prolongation, interpolated in time        */
/* between the parent's time levels (2nd order; 1st order while the       */
/* parent has no earlier level).  Patches of one depth exchange data where */
/* they meet: overlapping active cells take their mean after every step,  */
/* and a ghost point inside another patch's active region takes that      */
/* patch's value at every stage.  After the two steps of a depth every    */
/* coarse cell covered by one of its patches is overwritten by the        */
/* 4th-order Lagrange restriction (the mean where several cover it).      */
/* ---------------------------------------------------------------------- */

/* One patch.  Geometry as for z4c_box.  Patch 0 (the root): parent -1, bc
 * Z4C_BC_PERIODIC, Z4C_BC_SOMMERFELD or Z4C_BC_EQUATORIAL, obj -1.  Patches
 * >= 1: parent is the index of a patch listed before it; bc must be
 * Z4C_BC_COPY (ghosts come from the parent), n even, dx half the parent's,
 * and the lower faces on parent cell faces: F[d] is the parent active cell
 * index of that face, x0[d] = parent x0[d] + (F[d] - 1/4) * parent dx[d]
 * (checked); the 6-point stencils of every ghost must fall in the parent's
 * active cells.  obj: -1 for a fixed patch, else the index of the tracked
 * object the patch follows (z4c_hier_set_moving).  Equatorial symmetry
 * (Sec. 2.2.2, 2.4): with an equatorial root, a patch whose parent lies on
 * the symmetry plane and whose F[2] is 0 lies on it too; its prolongation
 * reads the parent's layers below the plane as mirror images (each field's z
 * parity), its own layers below the plane are the mirror images of its
 * active ones, and it never shifts in z.  All six arrays are
 * caller-owned device arrays of 25 fields with stride sf, distinct from
 * every other patch's: u the state (advanced in place), u_a, u_b, acc the
 * RK4 scratch, prev and cur the patch's time levels kept for its children
 * (any contents on entry; only the cells its children's prolongations read,
 * one cell wider for children that move, are written there). */
typedef struct z4c_level {
    int n[3];
    int ng;
    int bc;
    long sf;
    double dx[3];
    double x0[3];
    int F[3];
    double* u;
    double* u_a;
    double* u_b;
    double* acc;
    double* prev;
    double* cur;
    int parent;
    int obj;
} z4c_level;

/* Create a hierarchy of nlev (1..32) patches, at most 16 per depth,
 * advanced with root step dt0.  tile == NULL: the library default shape
 * with a persistent launch.  Allocates in device memory (Z4C_ENOMEM if that
 * fails):
 *   three ghost-shell buffers per patch >= 1, each 25 x (stored - active)
 *   doubles: the spatial prolongations of the parent's three time levels,
 *   which the ghost fill weights per stage time;
 *   the scratch of the separable prolongation: the x and y sums of two
 *   levels of every patch of the depth that needs most (25 x its parent-row
 *   window x its stored x-y extent, per level and pass). */
int z4c_hier_create(const z4c_level* levels, int nlev, const z4c_params* p, double dt0, const z4c_tile* tile,
                    void** hier);

/* Advance every patch by nsteps root steps on `stream`.  Ghosts of the
 * patches' states are not refreshed at the end (call apply_ghosts or read
 * the active cells).  use_graph: once every patch with children holds an
 * earlier time level, one root step is captured as a HIP graph on first use
 * and replayed (recaptured after a patch moved). */
int z4c_hier_advance(void* hier, int nsteps, int use_graph, void* stream);

/* Moving patches (Sec. 2.2.1): the patches with obj >= 0 follow the nobj
 * (1..16) punctures that start at xp (3 doubles per object, host).  Each
 * puncture is tracked on its object's deepest patch (exactly one patch of
 * the object at that depth) with dx^i/dt = -beta^i: Heun's method per step
 * of that patch, beta by 4-point Lagrange interpolation in each direction
 * from active cells.  After every root step z4c_hier_advance reads the
 * punctures back (a stream synchronisation) and, in patch order, shifts each
 * moving patch whose centre is more than two of its cells from its
 * puncture, per direction, by two cells toward it -- one parent cell, so F
 * moves by one and x0 by one parent dx; cells it covered before keep their
 * values, newly covered ones are prolonged from the parent, its children
 * keep their place in space (their F moves by -2).  A shift that would take
 * a patch's stencils out of its parent, or a puncture whose stencil leaves
 * its patch's active cells, fails with Z4C_EINVAL after that root step;
 * the patches the same regrid shifted before the refused one stay shifted
 * (and consistent), the refused one and those after it stay in place.
 * Allocates 80 bytes of device memory per object. */
int z4c_hier_set_moving(void* hier, int nobj, const double* xp);

/* Current punctures (xp, 3 doubles per object; may be NULL) and, if not
 * NULL, every patch's F and x0 (3 per patch); synchronises with the device. */
int z4c_hier_puncture(void* hier, double* xp, int* F, double* x0);

int z4c_hier_destroy(void* hier);

/* Static description of a status code, and the detail of the last failing
 * call on this thread. */
const char* z4c_strerror(int status);
const char* z4c_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* Z4C_H */
