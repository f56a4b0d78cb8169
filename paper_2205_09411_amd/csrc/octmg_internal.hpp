// Internal declarations of the octree multigrid library (host + device).
//
// Device data layout (per level, per right-hand side):
//   * blocks of N^D cells are stored one after another in the level's Morton
//     block order (block-major, Sec. 2.1);
//   * inside a block the cells are split by colour of the red-black
//     Gauss-Seidel smoother: [colour][N^D/2], colour = (i+j+k) & 1 (red = 0),
//     and within a colour x is compressed by two: q = (k*N + j)*(N/2) + i/2.
//     A red half-sweep then reads only black values and writes only red
//     values, so one smoothing step moves 24 B per cell in FP64 (read phi of
//     the other colour, read g, write phi) instead of twice that.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "octmg.h"

namespace octmg {

constexpr int kMaxLevels = 24;

// ------------------------------------------------------------ host tree
struct TreeLevel {
    int n = 0;    // cells per edge
    int Nb = 0;   // block edge
    int nb = 0;   // blocks per edge
    std::vector<int> pos;       // [nblocks][3], Morton order
    std::vector<uint8_t> leaf;  // [nblocks]
    std::vector<int> lut;       // nb^D -> block index or -1
    int nblocks() const { return (int)leaf.size(); }
};

struct Tree {
    int D = 0, N = 0, nsub = 0;
    bool adaptive = false;
    std::vector<TreeLevel> lv;  // coarsest first
};

// Builds the block tree: uniform or near-interface refinement, then 2:1
// balance over face, edge and corner neighbours (Sec. 2.1).  Returns false
// with a message on invalid input.
bool build_tree(const octmg_geom_desc &d, Tree *out, std::string *err);
// The tree of `old` after its leaves (canonical leaf order: level, then Morton)
// are flagged +1 refine (below max_level) or -1 coarsen (a family goes when
// all its children are flagged leaves above uniform_level), then balanced
// again.  The paper's setting: the mesh changes, the boundary does not.
bool adapt_tree(const octmg_geom_desc &d, const Tree &old, const int8_t *flags, Tree *out, std::string *err);

// Host evaluation of the geometry's level set (block-centre refinement test).
double lsf_host(const octmg_geom_desc &d, const double *params, const double *x);

// ------------------------------------------------------- device views
// One level as seen by a kernel.  Field pointers are the rhs-0 base; the
// kernel adds blockIdx.y * fstride for batched right-hand sides.
template <typename T>
struct LV {
    int n, nb, nblocks, nface;
    T dx2, inv_dx2;
    const int *lut;      // nb^D
    const int4 *pos;     // [nblocks] block coordinates
    const int4 *nbr;     // [2 nblocks] face neighbours x-,x+,y-,y+,z-,z+,pad,pad: block,
                         // -1 none on this level (coarser), -2 outside the domain
    const int *leaf;     // [nblocks]
    const int *map_off;  // [nblocks] offset of the block's record map, or -1
    const int *map;      // record index per cell (split order) or -1
    const T *rec;        // [nrec][8] = c(x-,x+,y-,y+,z-,z+) with cut links 0, diag, 1/diag
    const T *b;          // [nrec] moved boundary term (nullptr: homogeneous)
    const T *bcv;        // [2D][nface] domain face values (nullptr: homogeneous)
    T *phi, *g, *old;
    // prolonged black values that launch_prolong_gs leaves for the next
    // black half sweep (which then forms its cells' ghosts from them); set on
    // that sweep's view only (nullptr: ghosts from phi)
    T *own;
    long long fstride;
    const int *active;   // [nrhs] nonzero = right-hand side still iterating (nullptr: all)
    const int *lanes;    // [grid y] right-hand side of each grid row (nullptr: row = rhs)
    int order;           // workgroup -> block order of the 3D kernels (0 XCD ranges, 1 hardware)
    int neumann;         // bit 2 axis + (side > 0): zero-flux domain face (ghost = inside value)
    int pair_max;        // 3D launches of at most this many workgroups (blocks x grid rows) take the
                         // 512-thread variants (both colours staged at once); same results
};

// ---------------------------------------------------------- launches
// All launches are asynchronous on `s`; `nrhs` is the grid's y extent.
// D in {2,3}; N (block edge of the level) in {8,16}; Nc the coarse level's
// block edge.  Return hipSuccess or the launch error.
template <typename T>
hipError_t launch_gs_half(int D, int N, const LV<T> &L, const LV<T> &Lc, int color, int nrhs, hipStream_t s);
// 3D FP32 black half sweep with the mixed-precision update U.phi += e of
// every cell (both colours) of the level's leaf blocks.  keep = 0: every
// block is a leaf and the black values are not stored; keep = 1: they are
// stored and blocks with L.leaf[blk] = 0 are not updated.  N = 8 or 16
hipError_t launch_gs_half_update(int N, const LV<float> &L, const LV<float> &Lc, const LV<double> &U, int keep,
                                 int nrhs, hipStream_t s);
// phi_c is written to Lc.phi, or to Lc.old when `into_old` (adaptive trees:
// refinement-boundary ghosts of the fine level still read Lc.phi); then
// launch_copy_parents moves it to phi on parent blocks (and copies phi to
// old on leaf blocks).  In 3D phi_c is written to Lc.old in either case.
template <typename T>
hipError_t launch_restrict_fas(int D, int N, int Nc, const LV<T> &L, const LV<T> &Lc, int into_old, int nrhs,
                               hipStream_t s);
// A level of one 16^3 block covering the domain, in one workgroup per rhs:
// with restrict_to, [fas: the FAS right-hand side from old, which is also
// the starting iterate,] `steps` red-black sweeps, then the residual
// restricted into Lc (block edge Nc; into_old as in launch_restrict_fas);
// without, `steps` sweeps.  Same results as the separate launches.
template <typename T>
hipError_t launch_single_block(int Nc, const LV<T> &L, const LV<T> &Lc, int fas, int restrict_to, int steps, int into_old,
                               int nrhs, hipStream_t s);
template <typename T>
// leaves_only: only the leaf blocks' old <- phi (the parents' phi <- old is
// then left to launch_fas_gs with own_to_phi)
hipError_t launch_copy_parents(int D, int N, const LV<T> &L, int nrhs, hipStream_t s, int leaves_only = 0);
template <typename T>
hipError_t launch_restrict_rhs(int D, int N, int Nc, const LV<T> &L, const LV<T> &Lc, int nrhs, hipStream_t s);
template <typename T>
hipError_t launch_fas_rhs(int D, int N, const LV<T> &L, const LV<T> &Lc, int parents_only, int nrhs, hipStream_t s);
// 3D: the FAS right-hand side of level L (g <- L phi + g on parent blocks)
// fused with its first red half sweep; needs old = the restricted values on
// parent blocks and old = phi on leaf blocks (as the 3D restriction, plus
// launch_copy_parents on adaptive trees, leaves them).  own_to_phi: also
// set the black phi of parent blocks from old (when the restriction wrote
// old only).  Same results as launch_fas_rhs then launch_gs_half(colour 0).
template <typename T>
hipError_t launch_fas_gs(int D, int N, const LV<T> &L, const LV<T> &Lc, int own_to_phi, int nrhs, hipStream_t s);
template <typename T>
hipError_t launch_restrict_phi(int D, int N, int Nc, const LV<T> &L, const LV<T> &Lc, int nrhs, hipStream_t s);
template <typename T>
hipError_t launch_prolong(int D, int N, int Nc, const LV<T> &L, const LV<T> &Lc, int solution_mode, int nrhs,
                          hipStream_t s);
// 3D, V-cycle correction: launch_prolong (solution_mode 0) and the red half
// sweep after it in one launch; the black values stay unprolonged in phi
// and must be followed by launch_gs_half(colour 1) on a view with own = the
// same L.own (blocks with domain or refinement faces store their prolonged
// black values there).  Same results as the two separate launches.
template <typename T>
hipError_t launch_prolong_gs(int N, int Nc, const LV<T> &L, const LV<T> &Lc, int nrhs, hipStream_t s);
template <typename T>
// fas (3D): form the level's FAS right-hand side g + L phi from phi = old
// inside the solve (after launch_restrict_fas without launch_fas_rhs)
hipError_t launch_coarse_solve(int D, const LV<T> &L0, const double *M, const double *S, int fas, int nrhs,
                               hipStream_t s);
// The bottom of a FAS V-cycle (levels 0..top, 3D) in one cooperative launch.
constexpr int kMaxSmallLevels = 8;
template <typename T>
struct SmallLevels {
    LV<T> L[kMaxSmallLevels];
    int N[kMaxSmallLevels];
    int n_down, n_up, nrhs, into_old;
    const double *M, *S;
};
// P: device copy of the level table (read by the kernel while it runs);
// top: highest level of the fused part (1 <= top < kMaxSmallLevels)
template <typename T>
hipError_t launch_small_vcycle(const SmallLevels<T> *P, int top, int grid, hipStream_t s);
// co-resident workgroups of k_small_vcycle on the current device
template <typename T>
hipError_t small_vcycle_max_grid(int *grid);
// Residual norms: every workgroup combines its max |r| (bit pattern of a
// non-negative double; NaN as +Inf) with atomicMax into one of kNormSlots
// slots of its rhs, kNormStride words apart (slot = workgroup index mod
// kNormSlots), so that thousands of workgroups do not queue on one address;
// launch_norm_reduce then takes the max over the slots.
constexpr int kNormSlots = 16, kNormStride = 16;
constexpr long long norm_slot_words(int nrhs) { return (long long)nrhs * kNormSlots * kNormStride; }
// norm[r] = mapped[r] = max over the slots of rhs r, and the slots back to
// zero for the next norm (one workgroup)
hipError_t launch_norm_reduce(unsigned long long *slots, unsigned long long *norm, unsigned long long *mapped,
                              int nrhs, hipStream_t s);
// max |r| over the leaf blocks of a level into the norm slots `out`;
// phi_zero: residual of 0.
template <typename T>
hipError_t launch_residual_max(int D, int N, const LV<T> &L, const LV<T> &Lc, int phi_zero,
                               unsigned long long *out, int nrhs, hipStream_t s);
// leaf data <-> level fields (canonical leaf order); lb = leaf block ids.
hipError_t launch_scatter_leaf(int D, int N, const LV<double> &L, const int *lb, int nlb, const double *src,
                               long long src_stride, long long base, int field, int nrhs, hipStream_t s);
hipError_t launch_gather_leaf(int D, int N, const LV<double> &L, const int *lb, int nlb, double *dst,
                              long long dst_stride, long long base, int nrhs, hipStream_t s);
// whole-level canonical order <-> split layout (debug accessors)
hipError_t launch_level_copy(int D, int N, double *split, double *canon, int nblocks, int to_split, hipStream_t s);
// mixed precision: r64 = g - L phi on leaf blocks -> g32 = (float)r64,
// phi32 = 0 there, max |r64| into the norm slots `out`; and phi64 += phi32
// on leaf blocks.
// red_preset (3D): the red cells' FP32 correction is written as its first
// red half sweep from zero would leave it (the next FP32 V-cycle then starts
// with the black half sweep); otherwise the correction is zeroed
hipError_t launch_defect(int D, int N, const LV<double> &L, const LV<double> &Lc, LV<float> L32, const int *lb,
                         int nlb, unsigned long long *out, int nrhs, hipStream_t s, int red_preset = 0);
hipError_t launch_update(int D, int N, const LV<double> &L, LV<float> L32, const int *lb, int nlb, int nrhs,
                         hipStream_t s);
// b_i = sum over cut links of c_link * phi_b(point)
hipError_t launch_boundary_terms(int D, const int *meta, const double *cfull, int nrec, const double *vals,
                                 double *b64, float *b32, hipStream_t s);
hipError_t launch_fill(double *p, long long n, double v, hipStream_t s);
hipError_t launch_fillf(float *p, long long n, float v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, long long n, unsigned long long v, hipStream_t s);
// device-side convergence test of cycle *cbase + c of a graph solve: for
// every active rhs record its norm in hist[cycle][rhs] and freeze it once the
// norm is <= thresh[rhs] (or not finite, or at cycle max_cycles - 1); with
// advance > 0 (the last test of a chunk of that many cycles) *cbase then
// moves on by advance.  Cycles at or beyond max_cycles record nothing.
hipError_t launch_converge(const unsigned long long *norm, const double *thresh, int *active, double *hist, int c,
                           int nrhs, int *cbase, int max_cycles, int advance, hipStream_t s);
hipError_t launch_copy_d2f(const double *src, float *dst, long long n, hipStream_t s);
hipError_t launch_copy_f2d(const float *src, double *dst, long long n, hipStream_t s);
hipError_t launch_check_finite(const double *p, long long n, int *flag, hipStream_t s);
// phi of one level's leaf blocks of an adapted tree from the levels of the
// previous tree (Lold[nlev] and their block edges in device memory)
hipError_t launch_remap(int D, int N, const LV<double> &Ln, int il, const LV<double> *Lold, const int *nb_old,
                        const int *lb, int nlb, int nrhs, hipStream_t s);
// grad phi at the leaf cells of one level (Sec. 4.3: face differences, with
// (phi_b - phi_i)/(d dx) across cut links), out[rhs][n_leaf][3] at leaf
// offset base; inside_zero: cut cells with f(centre) < 0 get 0
hipError_t launch_gradient(int D, int N, const LV<double> &L, const LV<double> &Lc, const int *lb, int nlb,
                           const int *meta, const double *d6, const int *inside, const double *pb, int inside_zero,
                           double *out, long long out_stride, long long base, int nrhs, hipStream_t s);

// ------------------------------------------------------------- setup
// FP64 interface setup of one level (built without FMA contraction).
struct SetupLevel {
    int D, n, Nb, nblocks, nb;
    double dx, lo[3];
    const int4 *pos;
    const int *lut;
    const int *leaf;
    int lsf_kind, lsf_n;
    const double *lsf_params;  // device copy (host copy in the host passes)
    octmg_lsf_fn lsf_fn;       // OCTMG_LSF_CALLBACK (host passes only)
    void *lsf_user;
    double mask_L;             // mask_factor * sqrt(D) * dx
    double w_min;
    int nbisect, ngolden;
    const int *blocks = nullptr;  // if set: only these blocks (nlist of them)
    int nlist = 0;
};
// a block whose records an adapted geometry copies from its predecessor
struct ReuseBlock {
    int old_blk, new_blk, old_roff, new_roff, nrec, old_poff, new_poff, npt, old_moff, new_moff;
};
struct ReuseArrays {
    int *map, *meta, *inside;
    double *d6, *cfull, *rec8, *pts;
    float *rec8f;
};
hipError_t launch_reuse_records(const ReuseBlock *list, int nlist, int cpb, const ReuseArrays &o,
                                const ReuseArrays &n, hipStream_t s);
// pass 1: per block, the number of custom cells and of cut links (added to
// counts, which start at zero), and per cell a flag byte (0x80 | cut links
// for a custom cell, else 0; [nblocks][cells per block])
hipError_t launch_setup_count(const SetupLevel &S, int *counts /*[nblocks][2]*/, unsigned char *flags, hipStream_t s);
// pass 2: records in canonical order at the given per-block offsets; only
// the cells flagged by pass 1 are analysed again
hipError_t launch_setup_emit(const SetupLevel &S, const unsigned char *flags, const int *rec_off, const int *pt_off,
                             const int *map_off, int *map, int *meta /*[nrec][4]*/, double *d6,
                             double *cfull /*[nrec][6]*/, double *rec8, float *rec8f, double *pts,
                             int *inside /*[nrec]*/, hipStream_t s);
// the same two passes on the host, for a level set given as a host function
// (S holds host pointers; only the blocks of S.blocks if set)
void host_setup_count(const SetupLevel &S, int *counts);
void host_setup_emit(const SetupLevel &S, const int *rec_off, const int *pt_off, const int *map_off, int *map,
                     int *meta, double *d6, double *cfull, double *rec8, float *rec8f, double *pts, int *inside);
// coarsest grid: dense operator with domain ghosts folded in, then a
// row-equilibrated Gauss-Jordan inverse M and scales S (A^-1 = M diag(S)).
hipError_t launch_coarse_assemble(int D, int Nb, double dx, const int *map, const double *rec8, int neumann,
                                  double *A, hipStream_t s);
// mult: n doubles of workspace; fail: 1 when the operator is singular
hipError_t launch_gauss_jordan(int n, double *A, double *M, double *S, double *mult, int *fail, hipStream_t s);

// ---- lanes of a multi-rhs state (api.cpp), used by the serving engine.
// With device buffers these calls only enqueue work on `st`; the caller
// waits for the stream (an event) before reading norms or results.
octmg_status api_fail(octmg_status st, const std::string &msg);
int geom_device(octmg_geom g);
size_t lane_bytes(octmg_geom g, int precision);   // device bytes of one lane's fields
size_t state_fixed_bytes(octmg_geom g);           // device bytes of a state besides its lanes
// pinned control and mapped norm buffers of a lane state (once per state)
octmg_status lanes_prepare(octmg_state s);
// rhs of one lane from leaf-ordered values (host: staged and waited for;
// device: enqueued); zeroes its phi
octmg_status lane_load(octmg_state s, int lane, const double *src, int on_device, hipStream_t st);
// leaf-ordered phi of one lane into dst (host: waited for; device: enqueued)
octmg_status lane_store(octmg_state s, int lane, double *dst, int on_device, hipStream_t st);
// r0 and first convergence norm of the lanes flagged in `fresh`, enqueued
octmg_status lanes_begin(octmg_state s, const std::vector<int> &fresh, hipStream_t st);
void lanes_begin_norms(octmg_state s, std::vector<double> &r0, std::vector<double> &rk);
// one V-cycle of the flagged lanes plus their norms, asynchronously
octmg_status lanes_cycle(octmg_state s, const std::vector<int> &running, int kind, hipStream_t st);
// norms written by the last lanes_cycle (after its stream has passed it)
void lanes_norms(octmg_state s, std::vector<double> &out);

}  // namespace octmg
