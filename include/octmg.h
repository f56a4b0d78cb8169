/*
 * octmg.h -- C ABI of the octree geometric multigrid solver for Poisson's
 * equation with level-set-defined irregular Dirichlet boundaries, after
 * Teunissen & Schiavello, "Geometric multigrid method for solving Poisson's
 * equation on octree grids with irregular boundaries".
 *
 * Conventions for every entry point:
 *   - Every call returns octmg_status: 0 = OK, < 0 = error.  Nothing throws
 *     across the ABI.  The message of the last error on the calling thread is
 *     returned by octmg_last_error().
 *   - Handles are owned by the library and released by the matching
 *     *_destroy call.  Buffers passed in are borrowed for the duration of the
 *     call (host buffers) or until the given stream has passed the call
 *     (device buffers; on_device != 0).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work of a call is ordered on that stream.
 *   - A geometry is immutable after creation and may be shared by several
 *     states.  A state is used by one host thread at a time.
 *   - Leaf order ("canonical"): levels from coarse to fine, blocks of a level
 *     in Morton order (x bit lowest), cells of a block x-fastest.  Level
 *     order: the same without the leaf filter.
 *   - Levels are numbered 0 .. n_levels-1 from the coarsest grid (8^D cells,
 *     solved directly) to the finest.  Tree level l (root = 1 in the paper's
 *     numbering) is level index l - 1 + n_sub, where n_sub single-block
 *     levels sit below the root when block_n > coarse_n.
 *
 * Errors: OCTMG_ERR_INVALID for bad arguments (null handles, sizes out of
 * range, unsupported dim/block size); OCTMG_ERR_OOM when a device allocation
 * fails; OCTMG_ERR_HIP for any other HIP runtime failure (including no
 * device); OCTMG_ERR_NONFINITE when the rhs or boundary data holds NaN/Inf;
 * OCTMG_ERR_NOT_CONVERGED when a solve stops before rtol (the report is
 * filled); OCTMG_ERR_GEOMETRY for a tree the method cannot handle.
 */
#ifndef OCTMG_H
#define OCTMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OCTMG_OK = 0,
    OCTMG_ERR_INVALID = -1,
    OCTMG_ERR_OOM = -2,
    OCTMG_ERR_HIP = -3,
    OCTMG_ERR_NOT_CONVERGED = -4,
    OCTMG_ERR_NONFINITE = -5,
    OCTMG_ERR_GEOMETRY = -6,
    OCTMG_ERR_BUDGET = -7
} octmg_status;

/* level-set kinds (Sec. 3.1, eq. lsf-example) */
enum { OCTMG_LSF_NONE = 0,       /* no interface */
       OCTMG_LSF_SPHERES = 1,    /* union: f = min_m |x - c_m| - r_m; params [cx,cy,cz,r]*n */
       OCTMG_LSF_CYLINDER_Z = 2, /* f = |(x,y) - (cx,cy)| - r; params [cx,cy,r] */
       /* the sharp shapes of Sec. 4.2 (eqs. spheroid .. astroid) in
        * coordinates 2D: p = s (x - cx), q = s (y - cy); 3D, axisymmetric
        * about the z axis through (cx, cy): p = s (|(x - cx, y - cy)| - r0),
        * q = s (z - cz); params [cx, cy, cz, s, r0] (r0 unused in 2D);
        * |t|^(2/3) is evaluated as the cube root of t^2 computed with
        * + - * / only (bit-reproducible) */
       OCTMG_LSF_SPHEROID = 3,   /* sqrt(8 p^2 + q^2) - 1 */
       OCTMG_LSF_RHOMBUS = 4,    /* 8 |p| + |q| - 1.5 */
       OCTMG_LSF_HEART = 5,      /* p^2 + (q - |p|^(2/3))^2 - 1 */
       OCTMG_LSF_ASTROID = 6,    /* |p|^(2/3) / 0.8 + |q|^(2/3) / 1.5 - 0.8 */
       /* two electrodes (Sec. 4.3): min(dist(x, segment a-b) - r_rod,
        * |x - c| - r_sph); params [ax,ay,az, bx,by,bz, r_rod, cx,cy,cz, r_sph] */
       OCTMG_LSF_ELECTRODES = 7,
       /* any level set given as a host function (octmg_geom_desc.lsf_fn):
        * the setup (boundary mask, line search, unresolved-boundary search,
        * stencils) then runs on the host in FP64 with the same arithmetic as
        * the device setup of the built-in kinds; see octmg_lsf_fn */
       OCTMG_LSF_CALLBACK = 8 };

/* A user level set f(x) (Sec. 3.1: the interface is f = 0; cells with
 * f < 0 are inside).  x points to 3 coordinates (z = 0 in 2D).  Called on
 * the thread that runs octmg_plan_*, octmg_geom_create or octmg_geom_adapt,
 * one call at a time, about (1 + 2D) times per cell of every level plus a
 * few tens of times per cell near the interface (Sec. 3.2, Sec. 3.6.1).  It
 * must be deterministic.  As Sec. 3.6.1 notes, f need not be a distance
 * function, but the boundary mask assumes |grad f| describes f near its
 * zero contour. */
typedef double (*octmg_lsf_fn)(const double *x, void *user);
enum { OCTMG_REFINE_UNIFORM = 0, OCTMG_REFINE_NEAR_INTERFACE = 1 };
enum { OCTMG_FP64 = 0, OCTMG_MIXED = 1 };
enum { OCTMG_CYCLE_V = 0, OCTMG_CYCLE_FMG = 1 };
/* fields for the debug accessors */
enum { OCTMG_FIELD_PHI = 0, OCTMG_FIELD_G = 1, OCTMG_FIELD_OLD = 2 };
/* single method steps for kernel-level checks (octmg_debug_step) */
enum { OCTMG_STEP_HALF_SWEEP = 0,   /* arg = colour (0 red, 1 black) */
       OCTMG_STEP_SMOOTH = 1,       /* arg = number of red+black steps */
       OCTMG_STEP_RESTRICT_FAS = 2, /* level -> level-1 */
       OCTMG_STEP_PROLONG = 3,      /* level-1 -> level; arg = 1: solution mode */
       OCTMG_STEP_COARSE_SOLVE = 4, /* level ignored */
       OCTMG_STEP_RESTRICT_RHS = 5  /* level -> level-1, nested-iteration start */ };

/* Geometry description.  The domain is the cube [lo, lo+1]^D.
 * dim 2 or 3; block_n 8 or 16 cells per block edge; max_level >= 1 finest
 * tree level (root block = level 1, Sec. 2.1); refine_kind UNIFORM or
 * NEAR_INTERFACE (refine a block when |f(block centre)| < refine_width *
 * block width, then 2:1 balance over faces, edges and corners); eps_tol the
 * relative tolerance of the line search (Sec. 3.2, 1e-8 in the paper);
 * mask_factor the factor in L = mask_factor * sqrt(D) * dx of eq.
 * boundary-mask (1.5 in the paper); w_min the smallest width resolved on
 * coarse grids (Sec. 3.6.3; <= 0 disables); coarse_n the cells per edge of the
 * directly solved coarsest grid (8).  lsf_params is a host array read during
 * octmg_geom_create only.  lsf_fn and lsf_user (lsf_kind OCTMG_LSF_CALLBACK
 * only; lsf_params may then be NULL) must stay valid for the life of the
 * geometry and of the geometries adapted from it.
 * neumann_faces: bit f set makes domain face f (x-, x+, y-, y+, z-, z+ =
 * bits 0..5) a zero-flux face (ghost = the inside value), as on the sides of
 * the two-electrode problem of Sec. 4.3; the others are Dirichlet (values
 * from octmg_set_boundary).  At least one face or the interface must carry
 * Dirichlet data.  uniform_level: levels up to this one are complete
 * whatever refine_kind says (0: no such base). */
typedef struct octmg_geom_desc {
    int dim, block_n, max_level, refine_kind;
    int lsf_kind, lsf_n, coarse_n, neumann_faces;
    double refine_width, eps_tol, mask_factor, w_min;
    double lo[3];
    const double *lsf_params;
    int uniform_level, reserved;
    octmg_lsf_fn lsf_fn;
    void *lsf_user;
} octmg_geom_desc;

typedef struct octmg_geom_s *octmg_geom;
typedef struct octmg_state_s *octmg_state;

/* Context: the device, an optional allocator for every device buffer of the
 * geometries created in it and of their states (and of the temporaries of
 * their calls), and an optional tune-cache file for octmg_autotune.
 * alloc(bytes, device, user) returns device memory of at least `bytes` bytes
 * on `device` aligned to 256 bytes, or NULL (reported as OCTMG_ERR_OOM);
 * free(ptr, bytes, device, user) releases it; both may be called from the
 * thread of any call on those objects (a server's worker thread included)
 * and from octmg_*_destroy.  The callbacks must not call the library.
 * Without an allocator the library uses hipMalloc/hipFree.  The tune cache
 * is a text file of "<problem key> TAB <launch configuration> <ms>" lines
 * that octmg_autotune reads before timing and appends to after; the key
 * names the device, the tree's blocks per level, records, right-hand sides,
 * precision and solve options.  A geometry keeps its context alive
 * (reference counted): octmg_ctx_destroy may come before the geometries'
 * own destroy calls. */
typedef struct octmg_ctx_s *octmg_ctx;
typedef struct octmg_allocator {
    void *(*alloc)(size_t bytes, int device, void *user);
    void (*free)(void *ptr, size_t bytes, int device, void *user);
    void *user;
} octmg_allocator;
octmg_status octmg_ctx_create(int hip_device, const octmg_allocator *alloc_or_null, const char *tune_cache_path_or_null,
                              octmg_ctx *out);
void octmg_ctx_destroy(octmg_ctx c);

/* Launch configuration of a state's cycles.  Every choice gives the same
 * iterates, bit for bit; only the speed differs.
 *   block_order: which workgroup handles which block in the 3D level
 *     kernels -- 0: each of the 8 XCDs walks a contiguous Morton range of
 *     the level (face halos stay in that XCD's L2); 1: hardware order;
 *     2: on complete levels (nb^3 blocks) each XCD walks one Morton octant
 *     x-fastest (face neighbours a short distance apart in its dispatch
 *     order), elsewhere as 0.
 *   bottom_kind: 0 one launch per step and level; 1 the levels with at most
 *     bottom_max_blocks blocks run inside one cooperative launch (as
 *     octmg_state_set_fused_levels).
 *   graph_mode: the octmg_solve_opts.graph_mode recommended with it (a
 *     cooperative bottom cannot be captured: graph_mode 0 with bottom_kind 1).
 *   pair_max_blocks: 3D launches of at most this many workgroups (blocks x
 *     running right-hand sides) use 512 threads per block: restriction,
 *     FAS right-hand side and residual stage the two colours at the same
 *     time, prolongation and (16^3 blocks) the smoother give each thread
 *     half the cells.  Larger launches use 256 threads.  When the running
 *     right-hand sides number at most pair_max_blocks, a level made of one
 *     16^3 block below the finest level also runs its steps of a V-cycle in
 *     one 1024-thread workgroup per rhs (one launch per leg).  0: never.
 *     Every value gives the same iterates.  Default 1 << 30 (every launch).
 *   prolong_fused: 1 (default) runs the prolongation of a 3D V-cycle and
 *     the red half sweep after it as one launch (the black values are
 *     prolonged on the fly), 0 as two.  The same iterates either way.
 *   red_preset: 1 (default) lets the mixed-precision defect of a 3D tree
 *     write the FP32 correction's red cells on the finest level as the
 *     first red half sweep from zero leaves them, so the FP32 V-cycle starts
 *     there with the black half sweep; 0 zeroes the correction and runs that
 *     half sweep.  The same iterates either way.
 *   update_fused: 1 (default) lets the last (black) half sweep of each 3D
 *     level with leaf blocks in the mixed-precision FP32 correction's final
 *     V-cycle also add the correction to the FP64 solution on those blocks
 *     (phi += e, both colours), in place of a separate update launch; 0
 *     runs the two apart.  The same iterates either way. */
typedef struct octmg_launch_config {
    int block_order, bottom_kind, bottom_max_blocks, graph_mode, pair_max_blocks, prolong_fused, red_preset,
        update_fused;
} octmg_launch_config;
octmg_status octmg_state_set_launch(octmg_state s, const octmg_launch_config *c);
octmg_status octmg_state_get_launch(octmg_state s, octmg_launch_config *c);

/* Solve options (Sec. 2.2: V-cycle or FMG, N_down = N_up = 2). rtol is
 * relative to the max-norm residual of phi = 0 over the leaf cells.  The
 * solve stops with OCTMG_ERR_NOT_CONVERGED after max_cycles, or when the
 * residual ratio of successive cycles stays above 0.95 for 3 cycles.
 * graph_mode: 0 launches every kernel; 1 captures one cycle (with its
 * residual norm) in a HIP graph and replays it each cycle; 2 runs the
 * cycles as captured chunks, each cycle followed by a convergence test on
 * the device that stops the rhs it concerns (no stall test): a first chunk
 * of as many cycles as the state's previous solve took if that converged
 * (else all max_cycles of them when that is at most 16, else 8), then chunks of
 * one cycle until no rhs runs (the host reads the running flags between
 * chunks).  Results are identical in all modes.  Graph
 * modes capture on `stream` (or an internal stream if NULL) and need the
 * fused levels off; graphs are cached per state and rebuilt when the
 * smoothing counts or fused levels change. */
typedef struct octmg_solve_opts {
    int cycle_kind, max_cycles, zero_start, graph_mode;
    double rtol;
} octmg_solve_opts;

/* Solve report.  cycles, status, r0, r_final and history describe the
 * state as a whole (the largest residual over its right-hand sides).  The
 * four pointers are optional host arrays of n_rhs entries that the caller
 * sets (NULL: not filled): per right-hand side its status (OCTMG_OK when it
 * reached rtol, OCTMG_ERR_NOT_CONVERGED, OCTMG_ERR_NONFINITE), the cycles it
 * received (a converged rhs is frozen), the max-norm residual of phi = 0 and
 * the last residual. */
typedef struct octmg_solve_report {
    int cycles, status;
    double r0, r_final;
    double history[64]; /* max-norm residual after each cycle */
    int *rhs_status;
    int *rhs_cycles;
    double *rhs_r0;
    double *rhs_r_final;
} octmg_solve_report;

/* Message of the last failed call on this thread ("" if none). */
const char *octmg_last_error(void);
int octmg_version(void);

/* Host-only tree planning (Sec. 2.1), no device needed: per level
 * [n cells per edge, block edge, blocks, leaf blocks] into level_info
 * (caller provides 4 * 24 int64).  Same tree as octmg_geom_create. */
octmg_status octmg_plan_levels(const octmg_geom_desc *d, int *n_levels, int64_t *level_info);
/* Host-only: block positions and leaf flags of one level of the plan. */
octmg_status octmg_plan_blocks(const octmg_geom_desc *d, int level, int *pos, int *leaf);

/* Build the tree, run the FP64 interface setup on device `hip_device`
 * (boundary mask eq. boundary-mask, line search Sec. 3.2, unresolved
 * boundaries Sec. 3.6.3, stencils eq. lpl-2d-lsf, Sec. 3.6.2) and factor the
 * coarsest grid.  *out receives a new handle. */
octmg_status octmg_geom_create(const octmg_geom_desc *d, int hip_device, octmg_geom *out);
/* The same in a context (its device; hip_device is ignored), whose
 * allocator and tune cache serve the geometry, its states and the
 * geometries adapted from it. */
octmg_status octmg_geom_create_in(octmg_ctx ctx, const octmg_geom_desc *d, int hip_device, octmg_geom *out);
void octmg_geom_destroy(octmg_geom g);
/* info[0..7] = n_levels, n_leaf cells, n_interface points, n_domain face
 * points, custom-cell records (all levels), device bytes, tree blocks,
 * interface blocks. */
octmg_status octmg_geom_info(octmg_geom g, int64_t *info);
/* out[0..7] = n, block edge, blocks, leaf blocks, records, interface points,
 * face points per face, interface blocks of one level. */
octmg_status octmg_geom_level_info(octmg_geom g, int level, int64_t *out);
/* Host buffers: cell centres [n_leaf][3] and level index per leaf cell. */
octmg_status octmg_geom_leaf_coords(octmg_geom g, double *xyz, int *level);
/* Host buffer [n_interface][3]: the roots x0 of every cut link, ordered by
 * level, record (canonical cell order), link (x-,x+,y-,y+,z-,z+). */
octmg_status octmg_geom_iface_points(octmg_geom g, double *xyz);
/* Host buffer [n_domain][3]: domain face centres, ordered by level, face
 * (x-,x+,y-,y+,z-,z+), tangential cell index (lower axis fastest). */
octmg_status octmg_geom_domain_points(octmg_geom g, double *xyz);
/* Host buffers for one level: ids [nrec][3] = block, cell (canonical local
 * index), cut mask; d [nrec][6] relative distances (eq. relative-distance);
 * coef [nrec][8] = link coefficients (cut links included), diagonal, 0. */
octmg_status octmg_geom_records(octmg_geom g, int level, int *ids, double *d, double *coef);
octmg_status octmg_geom_block_positions(octmg_geom g, int level, int *pos, int *leaf);

/* Mesh adaptation (the paper's setting: the mesh changes often, the
 * boundary does not; Sec. 1 and Sec. 4.4).  flags[i] for the i-th leaf block
 * of g (canonical order: level, then Morton order within the level; the
 * blocks of octmg_geom_leaf_coords' cells, N^D cells each): +1 refine (below
 * max_level), -1 coarsen (a family of 2^D leaves goes when all are flagged
 * and their level is above uniform_level), 0 keep; then the tree is
 * balanced 2:1 again.  The result is a new geometry with g's level set and
 * descriptor.  reuse != 0: blocks with the same level, position and leaf
 * status keep g's stencil records, interface points and (if the coarsest
 * level is unchanged) the coarse inverse; only the other blocks run the
 * boundary detection and line search (Sec. 4.4: new refinement needs the
 * setup, removing refinement needs none).  The records equal those of a
 * setup from scratch, bit for bit.  stats (may be NULL): [blocks kept,
 * blocks set up, records kept, records computed].  g stays valid. */
octmg_status octmg_geom_adapt(octmg_geom g, const int8_t *flags, int reuse, octmg_geom *out, int64_t *stats);
/* phi of `from` carried to `to` (a state of a geometry adapted from
 * from's geometry, same n_rhs): unchanged cells are copied, cells of newly
 * refined blocks interpolated with the cell-centred (3/4, 1/4) weights from
 * the parent level, cells of coarsened blocks get the mean of their old
 * children.  A warm start for solves on the new mesh; rhs and boundary
 * values are set on `to` as usual.  Synchronises the stream. */
octmg_status octmg_state_remap(octmg_state from, octmg_state to, void *stream);

/* Fields for n_rhs right-hand sides on geometry g (kept alive by the state).
 * precision OCTMG_FP64, or OCTMG_MIXED: FP32 smoothing, transfers and ghost
 * fill inside an FP64 defect correction (FP64 residual, update, setup and
 * coarse solve). Solution and rhs start at zero; boundary data at zero. */
octmg_status octmg_state_create(octmg_geom g, int n_rhs, int precision, octmg_state *out);
void octmg_state_destroy(octmg_state s);
/* Smoothing steps per level visit (default 2 and 2). */
octmg_status octmg_state_set_smoothing(octmg_state s, int n_down, int n_up);
/* Levels with at most max_blocks blocks (3D) run the bottom of every
 * V-cycle -- the same smoothing, restriction, coarse solve and prolongation
 * steps (Sec. 2.2) -- inside one cooperative kernel launch with grid-wide
 * barriers between the steps; 0 (the default) launches every step
 * separately.  Results are identical either way. */
octmg_status octmg_state_set_fused_levels(octmg_state s, int max_blocks);
/* Dirichlet data shared by all right-hand sides: phi_b at every interface
 * point (octmg_geom_iface_points order; NULL = all zero) and at every domain
 * face point (octmg_geom_domain_points order; NULL = all zero).  The
 * interface term b_i = sum over cut links of c * phi_b is formed on the
 * device (Sec. 3.6.2: the value imposed at the boundary can change without
 * redoing the setup). */
octmg_status octmg_set_boundary(octmg_state s, const double *iface_vals, const double *domain_vals,
                                int on_device, void *stream);
/* Element type of the caller's rhs and solution buffers.  The solver
 * works in FP64 (in MIXED precision the inner cycles run in FP32, the
 * iterate is FP64); FP32 input is widened exactly, FP32 output is the FP64
 * solution rounded to nearest. */
enum { OCTMG_DTYPE_F64 = 0, OCTMG_DTYPE_F32 = 1 };
/* rhs g at leaf cells, [n_rhs][n_leaf] in canonical leaf order, elements
 * of type dtype.  OCTMG_ERR_NONFINITE if any value is NaN or Inf.
 * Synchronises the stream (host buffers are staged through device memory
 * that the call allocates and frees). */
octmg_status octmg_set_rhs(octmg_state s, const void *g, int dtype, int on_device, void *stream);
/* Initial guess / solution at leaf cells, [n_rhs][n_leaf], as for
 * octmg_set_rhs.  get_solution synchronises the stream. */
octmg_status octmg_set_solution(octmg_state s, const void *phi, int dtype, int on_device, void *stream);
octmg_status octmg_get_solution(octmg_state s, void *phi, int dtype, int on_device, void *stream);
octmg_status octmg_zero_solution(octmg_state s, void *stream);
/* Exactly one cycle: OCTMG_CYCLE_V (FAS V-cycle, Sec. 2.2) or
 * OCTMG_CYCLE_FMG (have_guess = 0 starts by restricting the rhs). In MIXED
 * precision one call is one outer defect-correction step around an FP32
 * cycle of that kind. */
octmg_status octmg_cycle(octmg_state s, int kind, int have_guess, void *stream);
/* Gradient of phi at every leaf cell centre (the field E = -grad phi of the
 * application in Sec. 4.3): on each cell face the difference to the
 * neighbour value or ghost over dx, or (phi_b - phi_i)/(d dx) across a cut
 * link (d the stored relative distance, phi_b the interface value); each
 * component is the mean of the cell's two faces.  inside_zero != 0: cells
 * with a cut link whose centre lies inside the interface (f < 0) report 0.
 * out[n_rhs][n_leaf][3] in canonical leaf order (host or device memory);
 * synchronises the stream. */
octmg_status octmg_gradient(octmg_state s, int inside_zero, double *out, int on_device, void *stream);
/* Max-norm of r = g - L phi (eq. residual) over the leaf cells, per rhs,
 * into the host array out[n_rhs] (synchronises the stream). phi_zero != 0:
 * residual of phi = 0. */
octmg_status octmg_residual_norm(octmg_state s, int phi_zero, double *out, void *stream);
/* Cycles until max|r| <= rtol * max|r(phi=0)| for every rhs. */
octmg_status octmg_solve(octmg_state s, const octmg_solve_opts *opts, void *stream, octmg_solve_report *rep);

/* For callers that cannot allocate device memory (work prepared for HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * octmg_solve for one right-hand side in FP64 from phi = 0, with every
 * field of the solve (phi, rhs and FAS rhs, restricted values, boundary
 * terms, norms, flags on all levels) in a fixed 64 MiB device array of the
 * library instead of a state.  Each device the call runs on holds its own
 * copy of the array until the process ends; the call allocates no device or
 * pinned host memory.  rhs [n_leaf] (canonical leaf order), iface_vals
 * [n_interface] and domain_vals [n_domain] (as octmg_set_boundary; NULL =
 * zero) are device pointers on g's device, as is the output phi [n_leaf].
 * opts as for octmg_solve except that graph_mode must be 0 and zero_start
 * is implied; rep (may be NULL) as for octmg_solve with n_rhs = 1.
 * Errors: OCTMG_ERR_INVALID when the geometry's fields do not fit the array
 * (about 24 B per cell of every level: up to 128^3 cells in 16^3 blocks),
 * OCTMG_ERR_NONFINITE for NaN/Inf input, OCTMG_ERR_NOT_CONVERGED (phi is
 * still written).  All calls on one device share the array: calls that
 * overlap on one device race and must be serialised by the caller; the
 * array keeps the last call's values, and each call clears what it reads.
 * Synchronises the stream. */
octmg_status octmg_solve_noalloc(octmg_geom g, const double *rhs, const double *iface_vals, const double *domain_vals,
                                 double *phi, const octmg_solve_opts *opts, void *stream, octmg_solve_report *rep);

/* Autotuner: solves the state's current problem from phi = 0 (opts, with
 * zero_start and graph_mode taken from each candidate) once to warm up and
 * `reps` times timed, under every candidate launch configuration (the three
 * block orders x {separate, separate in a per-cycle graph, cooperative
 * bottom up to 8 and to 64 blocks (3D)}, with the 512-thread variants on
 * every level, plus block order 0 {separate, per-cycle graph} with them on
 * none (3D), plus block order 0 with the solve replayed as captured chunks
 * of cycles (graph_mode 2) with the 512-thread
 * variants on every level and (3D) on none), then keeps the fastest in the
 * state and returns it.  ms[i] (if not NULL, room for 16) receives the mean
 * wall time per solve of candidate i, *n_candidates their number.
 * Afterwards phi holds the solution (the same under every candidate).
 * When the state's geometry was created in a context with a tune cache
 * that holds this problem's key, that configuration is applied without
 * timing (*n_candidates = 0, ms untouched, phi unchanged); otherwise the
 * winner is appended to the cache. */
octmg_status octmg_autotune(octmg_state s, const octmg_solve_opts *opts, int reps, void *stream,
                            octmg_launch_config *best, double *ms, int *n_candidates);

/* Profiling.  When enabled, each group of back-to-back red-black half
 * sweeps of the finest level (one level visit) is bracketed by HIP events
 * recorded on the stream it runs on, and the
 * smoother's cell updates are counted on all levels.  out[0] = finest-level
 * half sweeps timed, out[1] = their summed time in ms (synchronises
 * the recorded events), out[2] = smoother cell updates (all levels and
 * right-hand sides; a full red+black step counts each cell once), out[3] =
 * cells of the finest level.  Reading resets the counters. */
octmg_status octmg_profile_enable(octmg_state s, int enable);
octmg_status octmg_profile_read(octmg_state s, double *out);

/* Kernel-level access for parity checks: one level's field of one rhs in
 * canonical level order (host buffers, synchronous), and single steps of
 * the method on `level` (see OCTMG_STEP_*). FP64 fields of the state. */
octmg_status octmg_debug_get_field(octmg_state s, int level, int field, int rhs, double *out);
octmg_status octmg_debug_set_field(octmg_state s, int level, int field, int rhs, const double *in);
octmg_status octmg_debug_step(octmg_state s, int step, int level, int arg, void *stream);

/* ------------------------------------------------------------ serving
 * Independent solve requests, one right-hand side each, on geometries added
 * to the server (the method is built for solving many right-hand sides on
 * one set of boundaries, Sec. 1).  A worker thread batches the requests of
 * one geometry into the lanes of one multi-rhs state and admits waiting
 * requests between two V-cycles of the running ones (continuous batching);
 * each geometry's batch runs on its own stream, so batches of different
 * geometries overlap.  Every request is solved from phi = 0 with FAS
 * V(2,2) cycles and the tests of octmg_solve (rtol relative to the residual
 * of phi = 0, max_cycles, stall), and its result is identical to that of a
 * one-rhs octmg_solve of the same problem in the same precision.
 *
 * Device memory: states are held within hbm_budget_bytes, each charged
 * what it allocates: per lane 3 FP64 fields (plus 3 FP32 fields in MIXED
 * precision) per cell of every level and its norm and control words, per
 * state the boundary terms, face and interface values and one leaf-ordered
 * staging buffer; a geometry's state gets as many lanes as the budget and
 * max_lanes allow;
 * idle states of other geometries are released when a waiting geometry
 * needs room, and while one waits the others admit no new requests.  A request whose single lane
 * exceeds the budget completes with OCTMG_ERR_BUDGET.  Geometries are owned
 * by the caller and must outlive the server.
 *
 * Buffers are borrowed: rhs (n_leaf values in canonical leaf order) and
 * solution (n_leaf values) must stay valid until the request's result has
 * been polled; on_device selects device or host memory.  The solution is
 * written before the result is published (also for NOT_CONVERGED; not for
 * NONFINITE or BUDGET).  A rhs holding NaN or Inf completes with
 * OCTMG_ERR_NONFINITE.  Submit and poll are thread-safe and never block on
 * the GPU.  With device buffers the worker never waits for the GPU either
 * (every step of a request is enqueued on its geometry's stream and
 * completed through one polled event per geometry); host buffers are copied
 * synchronously by the worker. */
typedef struct octmg_server_s *octmg_server;
typedef struct octmg_server_opts {
    size_t hbm_budget_bytes;
    int max_lanes;  /* right-hand sides per batch, 1..4096 */
    int precision;  /* OCTMG_FP64 or OCTMG_MIXED */
    int max_cycles; /* per request, 1..64 */
    int reserved;
} octmg_server_opts;
typedef struct octmg_result {
    uint64_t id;
    int status; /* OCTMG_OK, OCTMG_ERR_NOT_CONVERGED, _NONFINITE, _BUDGET, _HIP */
    int cycles;
    double r0, r_final;             /* max-norm residuals of phi = 0 and of the result */
    double t_submit, t_admit, t_done; /* seconds on the server's monotonic clock */
} octmg_result;
typedef struct octmg_server_stats {
    uint64_t submitted, admitted, completed, failed;
    uint64_t states_created, states_released, cycles_launched, lane_cycles;
    uint64_t peak_bytes, bytes_in_use;
    double now; /* the server clock */
} octmg_server_stats;

octmg_status octmg_server_create(int device, const octmg_server_opts *opts, octmg_server *out);
/* Register a geometry with its Dirichlet data (host arrays as for
 * octmg_set_boundary; copied).  *slot names it in submissions. */
octmg_status octmg_server_add_geometry(octmg_server s, octmg_geom g, const double *iface_vals,
                                       const double *domain_vals, int *slot);
octmg_status octmg_server_submit(octmg_server s, int slot, const double *rhs, int rhs_on_device, double *solution,
                                 int solution_on_device, double rtol, uint64_t *id);
/* Up to cap finished results, in completion order (non-blocking). */
octmg_status octmg_server_poll(octmg_server s, octmg_result *done, int cap, int *n_done);
octmg_status octmg_server_get_stats(octmg_server s, octmg_server_stats *out);
/* Waits for queued and running requests to finish, then frees the server. */
void octmg_server_destroy(octmg_server s);

#ifdef __cplusplus
}
#endif
#endif /* OCTMG_H */
