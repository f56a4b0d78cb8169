// C ABI of the octree multigrid solver: geometry (tree + FP64 interface
// setup + coarse inverse, device resident), states (fields per right-hand
// side), and the FAS V-cycle / FMG engine that drives the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "octmg_internal.hpp"

using namespace octmg;

namespace {

thread_local std::string g_last_error;

octmg_status fail(octmg_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

#define HIPCK(call)                                                                                   \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) {                                                                       \
            return fail(e_ == hipErrorOutOfMemory ? OCTMG_ERR_OOM : OCTMG_ERR_HIP,                   \
                        std::string(#call) + ": " + hipGetErrorString(e_));                           \
        }                                                                                             \
    } while (0)

#define STCK(call)                        \
    do {                                  \
        octmg_status s_ = (call);         \
        if (s_ != OCTMG_OK) return s_;    \
    } while (0)

// device allocation owned by a geometry, a state or a call: hipMalloc, or
// the allocator of the geometry's context
struct DevPool {
    const octmg_allocator *a = nullptr;
    int device = 0;
    std::vector<std::pair<void *, size_t>> ptrs;
    size_t bytes = 0;
    DevPool() = default;
    DevPool(const octmg_allocator *alloc, int dev) : a(alloc), device(dev) {}
    DevPool(const DevPool &) = delete;
    DevPool &operator=(const DevPool &) = delete;
    ~DevPool() {
        for (auto &p : ptrs) {
            if (a) a->free(p.first, p.second, device, a->user);
            else (void)hipFree(p.first);
        }
    }
    template <typename T>
    hipError_t alloc(T **p, size_t n) {
        *p = nullptr;
        if (n == 0) return hipSuccess;
        void *q = nullptr;
        const size_t nb = n * sizeof(T);
        if (a) {
            q = a->alloc(nb, device, a->user);
            if (!q) return hipErrorOutOfMemory;
        } else {
            hipError_t e = hipMalloc(&q, nb);
            if (e != hipSuccess) return e;
        }
        ptrs.push_back({q, nb});
        bytes += nb;
        *p = (T *)q;
        return hipSuccess;
    }
};

struct GeomLevel {
    int n = 0, Nb = 0, nb = 0, nblocks = 0, nleaf = 0, cpb = 0, nface = 0;
    double dx = 0;
    std::vector<int> leaf_blocks;
    long long leaf_base = 0;   // canonical offset of the level's first leaf cell
    int nrec = 0, n_iface_blocks = 0;
    long long npts = 0, pt_base = 0;
    int4 *d_pos = nullptr, *d_nbr = nullptr;
    int *d_lut = nullptr, *d_leaf = nullptr, *d_map_off = nullptr, *d_map = nullptr;
    int *d_leaf_blocks = nullptr, *d_meta = nullptr, *d_inside = nullptr;
    double *d_rec8 = nullptr, *d_d6 = nullptr, *d_cfull = nullptr, *d_pts = nullptr;
    float *d_rec8f = nullptr;
    // per block: records and interface points, their offsets, record-map offset
    std::vector<int> h_nrec, h_npt, h_rec_off, h_pt_off, h_map_off;
};

}  // namespace

// device, allocator and tune cache shared by the geometries created in it
struct octmg_ctx_s {
    int device = 0;
    octmg_allocator alloc{};
    bool has_alloc = false;
    std::string tune_path;
    int refs = 1;
    const octmg_allocator *allocator() const { return has_alloc ? &alloc : nullptr; }
};

struct octmg_geom_s {
    octmg_ctx ctx = nullptr;  // may be null: hipMalloc, no tune cache
    octmg_geom_desc desc{};
    std::vector<double> params;
    int device = 0;
    Tree tree;
    std::vector<GeomLevel> L;
    long long n_leaf = 0, n_pts = 0, n_dom = 0, n_rec = 0, n_iface_blocks = 0;
    double *d_M = nullptr, *d_S = nullptr;
    DevPool pool;
    int refs = 1;
    const octmg_allocator *allocator() const { return ctx ? ctx->allocator() : nullptr; }
};

namespace {

struct Fields64 {
    double *phi = nullptr, *g = nullptr, *old = nullptr, *b = nullptr, *bcv = nullptr;
    double *bp = nullptr;  // prolonged black values of a fused prolongation (launch_prolong_gs)
    double *pb = nullptr;  // phi_b at the level's interface points (for the gradient)
};
struct Fields32 {
    float *phi = nullptr, *g = nullptr, *old = nullptr;
    float *bp = nullptr;
};

}  // namespace

struct Profile {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<int> launches;  // half sweeps inside each pending pair
    std::vector<hipEvent_t> spare;
    double updates = 0.0;
    hipEvent_t get() {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    ~Profile() {
        for (auto &p : pending) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
        for (auto e : spare) (void)hipEventDestroy(e);
    }
};

struct octmg_state_s {
    octmg_geom geom = nullptr;
    Profile *prof = nullptr;
    int nrhs = 1, precision = OCTMG_FP64, n_down = 2, n_up = 2;
    std::vector<Fields64> f64;
    std::vector<Fields32> f32;
    std::vector<long long> stride;  // per level: cells per rhs
    unsigned long long *d_norm = nullptr;
    unsigned long long *d_norm_slots = nullptr;  // per-rhs slots the norm kernels combine into
    // the slots are zero (left so by the last reduction); false from the
    // first norm kernel until the reduction, so that a norm cut short by an
    // error is followed by a clearing fill
    bool norm_slots_clean = false;
    int *d_flag = nullptr;
    // launch set: d_active[0, nrhs) = 1 while a right-hand side iterates;
    // d_active[nrhs, nrhs + n_launch) = the iterating right-hand sides, which
    // the kernels' grid rows walk (all of them: no list, grid y = rhs)
    int *d_active = nullptr;
    std::vector<int> active_host;              // flags last uploaded
    std::vector<int> lanes_host;               // list last uploaded
    int n_launch = 1;                          // grid rows of every per-rhs launch
    unsigned long long *h_norm = nullptr;      // pinned, host-mapped copy of d_norm
    unsigned long long *h_norm_dev = nullptr;  // device view of h_norm
    // serving lanes (lanes_prepare): pinned control uploads, two per pass of
    // the server, and host-mapped norms of newly admitted lanes [2][nrhs]
    // (residual of phi = 0, first defect)
    int *h_ctrl = nullptr;
    int ctrl_turn = 0;
    unsigned long long *h_begin = nullptr;
    unsigned long long *h_begin_dev = nullptr;
    std::vector<double> r0_cache;              // residual of phi = 0 (valid while !r0_dirty)
    bool r0_dirty = true;
    int block_order = 0;                       // LV::order of every level
    int tuned_graph = 0;                       // graph mode recommended by octmg_autotune
    int fused_max_blocks = 0;                  // levels with <= this many blocks run fused (0: off)
    int pair_max_blocks = 1 << 30;             // LV::pair_max of every level
    int prolong_fused = 1;                     // V-cycle prolongation fused with the next red half sweep (3D)
    int red_preset = 1;                        // mixed precision: first red half sweep inside the defect (3D)
    int update_fused = 1;                      // mixed precision: FP64 update inside the last black half sweep (3D)
    int cycle_hint = 0;                        // cycles of the last solve (first chunk of graph_mode 2), 0: none
    int fused_top = 0;                         // highest fused level (0: none)
    int fused_grid64 = 0, fused_grid32 = 0;    // co-resident workgroups of the fused kernel
    SmallLevels<double> *d_small64 = nullptr;  // device copies of the fused level tables
    SmallLevels<float> *d_small32 = nullptr;
    // captured solves: key -> executable graph (see solve_impl)
    std::vector<std::pair<long long, hipGraphExec_t>> graphs;
    hipStream_t own_stream = nullptr;          // capture stream when the caller passes NULL
    double *d_thresh = nullptr;                // [nrhs] rtol * r0 for device-side convergence
    double *d_hist = nullptr;                  // [64][nrhs] residual history of a graph solve
    int *d_cbase = nullptr;                    // first cycle number of the chunk a graph solve replays
    DevPool pool;
};

namespace {

int cells_per_block(int D, int Nb) { return D == 3 ? Nb * Nb * Nb : Nb * Nb; }

void release_ctx(octmg_ctx c) {
    if (c && --c->refs == 0) delete c;
}

void release_geom(octmg_geom g) {
    if (!g) return;
    if (--g->refs == 0) {
        (void)hipSetDevice(g->device);
        octmg_ctx c = g->ctx;
        delete g;  // frees through the context's allocator
        release_ctx(c);
    }
}

// ------------------------------------------------------------ level views
LV<double> lv64(const octmg_state_s *s, int il) {
    LV<double> v{};
    if (il < 0) return v;
    const GeomLevel &G = s->geom->L[il];
    v.n = G.n;
    v.nb = G.nb;
    v.nblocks = G.nblocks;
    v.nface = G.nface;
    v.dx2 = G.dx * G.dx;
    v.inv_dx2 = 1.0 / (G.dx * G.dx);
    v.lut = G.d_lut;
    v.pos = G.d_pos;
    v.nbr = G.d_nbr;
    v.leaf = G.d_leaf;
    v.map_off = G.nrec ? G.d_map_off : nullptr;
    v.map = G.d_map;
    v.rec = G.d_rec8;
    v.b = s->f64[il].b;
    v.bcv = s->f64[il].bcv;
    v.phi = s->f64[il].phi;
    v.g = s->f64[il].g;
    v.old = s->f64[il].old;
    v.fstride = s->stride[il];
    v.active = s->d_active;
    v.lanes = s->n_launch < s->nrhs ? s->d_active + s->nrhs : nullptr;
    v.order = s->block_order;
    v.neumann = s->geom->desc.neumann_faces;
    v.pair_max = s->pair_max_blocks;
    return v;
}

LV<float> lv32(const octmg_state_s *s, int il) {
    LV<float> v{};
    if (il < 0) return v;
    const GeomLevel &G = s->geom->L[il];
    v.n = G.n;
    v.nb = G.nb;
    v.nblocks = G.nblocks;
    v.nface = G.nface;
    v.dx2 = (float)(G.dx * G.dx);
    v.inv_dx2 = (float)(1.0 / (G.dx * G.dx));
    v.lut = G.d_lut;
    v.pos = G.d_pos;
    v.nbr = G.d_nbr;
    v.leaf = G.d_leaf;
    v.map_off = G.nrec ? G.d_map_off : nullptr;
    v.map = G.d_map;
    v.rec = G.d_rec8f;
    v.b = nullptr;    // the correction equation has homogeneous boundary data
    v.bcv = nullptr;
    v.phi = s->f32[il].phi;
    v.g = s->f32[il].g;
    v.old = s->f32[il].old;
    v.fstride = s->stride[il];
    v.active = s->d_active;
    v.lanes = s->n_launch < s->nrhs ? s->d_active + s->nrhs : nullptr;
    v.order = s->block_order;
    v.neumann = s->geom->desc.neumann_faces;
    v.pair_max = s->pair_max_blocks;
    return v;
}

template <typename T>
LV<T> lvT(const octmg_state_s *s, int il);
template <>
LV<double> lvT<double>(const octmg_state_s *s, int il) { return lv64(s, il); }
template <>
LV<float> lvT<float>(const octmg_state_s *s, int il) { return lv32(s, il); }

// ---------------------------------------------------------- cycle engine
template <typename T>
struct Engine {
    const octmg_state_s *s;
    hipStream_t st;
    int D() const { return s->geom->tree.D; }
    int Nb(int il) const { return s->geom->L[il].Nb; }

    // The half sweeps of one level visit run back to back; when profiling,
    // one event pair brackets the whole group on the finest level and the
    // group's time is shared evenly by its launches.
    // fas_first: the first red half sweep also forms the level's FAS
    // right-hand side (see restrict_only)
    // after_prolong: the first red half sweep has run inside the fused
    // prolongation (prolong_fused); the first black one takes its cells' own
    // values for the ghosts from the prolonged black values it left.  The
    // timed group then holds the remaining 2 steps - 1 half sweeps.
    // red_preset: the first red half sweep has run inside the mixed-precision
    // defect (the correction starts from zero there); it is skipped.
    // update_last (FP32 correction of a mixed-precision solve, upd set): the
    // last (black) half sweep also adds the correction to the FP64 solution
    // on the level's leaf blocks (k_gs_half3_update); it stays outside the
    // timed group.
    octmg_status smooth(int il, int steps, bool fas_first = false, bool after_prolong = false,
                        bool red_preset = false, bool update_last = false) {
        Profile *P = s->prof;
        const int plain = 2 * steps - (after_prolong || red_preset ? 1 : 0) - (update_last && steps > 0 ? 1 : 0);
        const bool timed = P && P->on && il == (int)s->geom->L.size() - 1 && plain > 0;
        hipEvent_t a = nullptr, b = nullptr;
        if (timed) {
            a = P->get();
            b = P->get();
            HIPCK(hipEventRecord(a, st));
        }
        for (int k = 0; k < steps; k++)
            for (int color = 0; color < 2; color++) {
                if ((after_prolong || red_preset) && k == 0 && color == 0) continue;
                const bool upd_here = update_last && k == steps - 1 && color == 1;
                if (upd_here && timed) HIPCK(hipEventRecord(b, st));
                if (fas_first && k == 0 && color == 0) {
                    HIPCK(launch_fas_gs<T>(D(), Nb(il), lvT<T>(s, il), lvT<T>(s, il - 1),
                                           s->geom->tree.adaptive ? 1 : 0, s->n_launch, st));
                } else {
                    LV<T> v = lvT<T>(s, il);
                    if (after_prolong && k == 0) v.own = bp_of(il);
                    if (upd_here) {
                        HIPCK(sweep_update(il, v));
                        upd_levels |= 1ull << il;
                    } else {
                        HIPCK(launch_gs_half<T>(D(), Nb(il), v, lvT<T>(s, il - 1), color, s->n_launch, st));
                    }
                }
                if (P && P->on) {
                    const GeomLevel &G = s->geom->L[il];
                    P->updates += 0.5 * (double)G.nblocks * G.cpb * s->n_launch;
                }
            }
        if (timed) {
            if (!(update_last && steps > 0)) HIPCK(hipEventRecord(b, st));
            P->pending.push_back({a, b});
            P->launches.push_back(plain);
        }
        return OCTMG_OK;
    }
    // FP32 correction of a mixed-precision solve: the last half sweep of each
    // level with leaves in the final V-cycle adds the correction to the FP64
    // solution there (mixed_correct sets upd); upd_levels: the levels it did
    bool upd = false;
    unsigned long long upd_levels = 0;
    hipError_t sweep_update(int il, const LV<T> &v);
    T *bp_of(int il) const;
    // the prolongation into il and its first red half sweep in one launch:
    // 3D levels smoothed by separate launches, with post-smoothing
    bool prolong_fusable(int il) const {
        return D() == 3 && s->prolong_fused && s->n_up >= 1 && !single_block(il) && bp_of(il) != nullptr &&
               (Nb(il) == 16 || (Nb(il) == 8 && Nb(il - 1) == 8));
    }
    octmg_status prolong_gs(int il) {
        LV<T> v = lvT<T>(s, il);
        v.own = bp_of(il);
        HIPCK(launch_prolong_gs<T>(Nb(il), Nb(il - 1), v, lvT<T>(s, il - 1), s->n_launch, st));
        Profile *P = s->prof;
        if (P && P->on) {
            const GeomLevel &G = s->geom->L[il];
            P->updates += 0.5 * (double)G.nblocks * G.cpb * s->n_launch;
        }
        return OCTMG_OK;
    }
    octmg_status half_sweep(int il, int color) {
        HIPCK(launch_gs_half<T>(D(), Nb(il), lvT<T>(s, il), lvT<T>(s, il - 1), color, s->n_launch, st));
        return OCTMG_OK;
    }
    // FAS restriction il -> il-1, then g_c = L_c phi_c + r_c, old_c = phi_c
    // (done: the restriction itself has run, inside single_block_down)
    octmg_status restrict_fas(int il, bool done = false) {
        const int adaptive = s->geom->tree.adaptive ? 1 : 0;
        if (!done)
            HIPCK(launch_restrict_fas<T>(D(), Nb(il), Nb(il - 1), lvT<T>(s, il), lvT<T>(s, il - 1), adaptive, s->n_launch,
                                         st));
        if (adaptive) HIPCK(launch_copy_parents<T>(D(), Nb(il - 1), lvT<T>(s, il - 1), s->n_launch, st));
        HIPCK(launch_fas_rhs<T>(D(), Nb(il - 1), lvT<T>(s, il - 1), lvT<T>(s, il - 2), 1, s->n_launch, st));
        return OCTMG_OK;
    }
    // FAS restriction il -> il-1 without the right-hand side, which the first
    // half sweep of il-1 (smooth with fas_first), or the coarse solve, then
    // forms from old.  On adaptive trees the restriction writes old only and
    // leaf blocks copy phi to old here; the parents' phi is set by that
    // half sweep (the coarse solve overwrites it).
    octmg_status restrict_only(int il, bool done = false) {
        const int adaptive = s->geom->tree.adaptive ? 1 : 0;
        if (!done)
            HIPCK(launch_restrict_fas<T>(D(), Nb(il), Nb(il - 1), lvT<T>(s, il), lvT<T>(s, il - 1), adaptive, s->n_launch,
                                         st));
        if (adaptive) HIPCK(launch_copy_parents<T>(D(), Nb(il - 1), lvT<T>(s, il - 1), s->n_launch, st, 1));
        return OCTMG_OK;
    }
    // whether coarse level lc of a V-cycle whose levels up to ft run fused
    // gets its FAS right-hand side from its first half sweep (3D, lc smoothed
    // by separate launches of the 512-lane kernels)
    bool fas_in_sweep(int lc, int ft) const {
        return D() == 3 && s->n_down >= 1 && lc > ft && lc >= 1 &&
               (long long)s->geom->L[lc].nblocks * s->n_launch <= s->pair_max_blocks;
    }
    // whether level il is one 16^3 block covering the domain, below the
    // finest level (whose sweeps bench.py's profiling events time), with the
    // colour-pair kernels enabled for its launches: then its steps of a
    // V-cycle run in one workgroup per rhs (launch_single_block)
    bool single_block(int il) const {
        const GeomLevel &G = s->geom->L[il];
        return D() == 3 && il >= 1 && il < (int)s->geom->L.size() - 1 && G.Nb == 16 && G.nb == 1 && G.nblocks == 1 &&
               s->n_launch <= s->pair_max_blocks;
    }
    void count_updates(int il, int steps) {
        Profile *P = s->prof;
        if (P && P->on) P->updates += (double)steps * s->geom->L[il].nblocks * s->geom->L[il].cpb * s->n_launch;
    }
    // the down leg on such a level: [FAS rhs,] n_down sweeps and the
    // restriction into il-1 (what smooth + launch_restrict_fas do)
    octmg_status single_block_down(int il, bool fas) {
        const int adaptive = s->geom->tree.adaptive ? 1 : 0;
        HIPCK(launch_single_block<T>(Nb(il - 1), lvT<T>(s, il), lvT<T>(s, il - 1), fas ? 1 : 0, 1, s->n_down, adaptive,
                                     s->n_launch, st));
        count_updates(il, s->n_down);
        return OCTMG_OK;
    }
    octmg_status single_block_up(int il) {
        HIPCK(launch_single_block<T>(Nb(il - 1), lvT<T>(s, il), lvT<T>(s, il - 1), 0, 0, s->n_up, 0, s->n_launch, st));
        count_updates(il, s->n_up);
        return OCTMG_OK;
    }
    octmg_status restrict_rhs(int il) {
        LV<T> c = lvT<T>(s, il - 1);
        const long long n = s->stride[il - 1] * s->nrhs;
        HIPCK(fill(c.phi, n));
        HIPCK(fill(c.old, n));
        HIPCK(launch_restrict_rhs<T>(D(), Nb(il), Nb(il - 1), lvT<T>(s, il), c, s->n_launch, st));
        return OCTMG_OK;
    }
    octmg_status prolong(int il, int solution_mode) {
        HIPCK(launch_prolong<T>(D(), Nb(il), Nb(il - 1), lvT<T>(s, il), lvT<T>(s, il - 1), solution_mode, s->n_launch, st));
        return OCTMG_OK;
    }
    octmg_status coarse_solve(int fas = 0) {
        HIPCK(launch_coarse_solve<T>(D(), lvT<T>(s, 0), s->geom->d_M, s->geom->d_S, fas, s->n_launch, st));
        return OCTMG_OK;
    }
    hipError_t fill(T *p, long long n);
    octmg_status sync_down() {
        if (!s->geom->tree.adaptive) return OCTMG_OK;
        for (int il = (int)s->geom->L.size() - 1; il > 0; il--)
            HIPCK(launch_restrict_phi<T>(D(), Nb(il), Nb(il - 1), lvT<T>(s, il), lvT<T>(s, il - 1), s->n_launch, st));
        return OCTMG_OK;
    }
    octmg_status fused(int top);
    // FAS V-cycle with top level `top` (Sec. 2.2).  Levels up to fused_top
    // (few blocks each) run in one cooperative launch with the same steps.
    // top_red_preset: the top level's first red half sweep has already run
    // (inside the mixed-precision defect, see mixed_red_preset)
    octmg_status vcycle(int top, bool top_red_preset = false) {
        const int ft = std::min(top, s->fused_top);
        bool fas_pending = false;
        // the coarsest level's FAS right-hand side is formed inside the solve (3D)
        const bool fas_coarse = ft == 0 && D() == 3;
        for (int il = top; il > ft; il--) {
            const bool sb = single_block(il);
            STCK(sb ? single_block_down(il, fas_pending)
                    : smooth(il, s->n_down, fas_pending, false, top_red_preset && il == top));
            fas_pending = fas_in_sweep(il - 1, ft);
            STCK(fas_pending || (il == 1 && fas_coarse) ? restrict_only(il, sb) : restrict_fas(il, sb));
        }
        if (ft >= 1) STCK(fused(ft));
        else STCK(coarse_solve(fas_coarse && top >= 1 ? 1 : 0));
        // in the final V-cycle (top = the finest level) each level's leaf
        // values are final after its post-smoothing: its last half sweep may
        // carry the FP64 update
        const bool last = upd && top == (int)s->geom->L.size() - 1;
        for (int il = std::max(ft, 0) + 1; il <= top; il++) {
            const bool ul = last && s->geom->L[il].nleaf > 0 && !single_block(il) && il < 64 &&
                            (Nb(il) == 8 || Nb(il) == 16);
            if (prolong_fusable(il)) {
                STCK(prolong_gs(il));
                STCK(smooth(il, s->n_up, false, true, false, ul));
                continue;
            }
            STCK(prolong(il, 0));
            STCK(single_block(il) ? single_block_up(il) : smooth(il, s->n_up, false, false, false, ul));
        }
        return OCTMG_OK;
    }
    // FMG (Sec. 2.2): restrict to the coarsest grid, solve, then a V-cycle on
    // each finer level after prolongating its correction.
    octmg_status fmg(int have_guess) {
        const int top = (int)s->geom->L.size() - 1;
        for (int il = top; il > 0; il--) STCK(have_guess ? restrict_fas(il) : restrict_rhs(il));
        STCK(coarse_solve());
        for (int il = 1; il <= top; il++) {
            STCK(prolong(il, have_guess ? 0 : 1));
            STCK(vcycle(il));
        }
        return OCTMG_OK;
    }
    // sync: leave the coarse copies of leaf values current (not needed when
    // the iterate is a correction that only the leaves pass on)
    octmg_status cycle(int kind, int have_guess, bool sync = true, bool red_preset = false) {
        const int top = (int)s->geom->L.size() - 1;
        STCK(kind == OCTMG_CYCLE_FMG ? fmg(have_guess) : vcycle(top, red_preset));
        return sync ? sync_down() : OCTMG_OK;
    }
};

template <>
octmg_status Engine<double>::fused(int top) {
    int most = 16;
    for (int il = 0; il <= top; il++) most = std::max(most, s->geom->L[il].nblocks);
    const int grid = std::max(1, std::min(s->fused_grid64, most * s->nrhs));
    HIPCK(launch_small_vcycle<double>(s->d_small64, top, grid, st));
    return OCTMG_OK;
}
template <>
octmg_status Engine<float>::fused(int top) {
    int most = 16;
    for (int il = 0; il <= top; il++) most = std::max(most, s->geom->L[il].nblocks);
    const int grid = std::max(1, std::min(s->fused_grid32, most * s->nrhs));
    HIPCK(launch_small_vcycle<float>(s->d_small32, top, grid, st));
    return OCTMG_OK;
}
template <>
hipError_t Engine<double>::sweep_update(int, const LV<double> &) { return hipErrorInvalidValue; }
template <>
hipError_t Engine<float>::sweep_update(int il, const LV<float> &v) {
    // below the finest level of an adaptive tree parent blocks and finer
    // levels' refinement ghosts still read the black correction
    const int keep = s->geom->tree.adaptive && il + 1 < (int)s->geom->L.size() ? 1 : 0;
    return launch_gs_half_update(Nb(il), v, lvT<float>(s, il - 1), lv64(s, il), keep, s->n_launch, st);
}
template <>
double *Engine<double>::bp_of(int il) const { return s->f64[il].bp; }
template <>
float *Engine<float>::bp_of(int il) const { return s->f32.empty() ? nullptr : s->f32[il].bp; }
template <>
hipError_t Engine<double>::fill(double *p, long long n) { return launch_fill(p, n, 0.0, st); }
template <>
hipError_t Engine<float>::fill(float *p, long long n) { return launch_fillf(p, n, 0.0f, st); }

// synced: phi's coarse copies are already current (right after a cycle)
// The norms land in d_norm and in the mapped host buffer.
// mapped: host-mapped norm buffer to write (default: the state's h_norm)
octmg_status residual_norm_dev(octmg_state s, int phi_zero, hipStream_t st, bool synced = false,
                               unsigned long long *mapped = nullptr) {
    if (!s->norm_slots_clean) HIPCK(launch_fill_u64(s->d_norm_slots, norm_slot_words(s->nrhs), 0ull, st));
    s->norm_slots_clean = false;
    if (!phi_zero && !synced) {
        Engine<double> e{s, st};
        STCK(e.sync_down());
    }
    const int D = s->geom->tree.D;
    for (int il = 0; il < (int)s->geom->L.size(); il++) {
        const GeomLevel &G = s->geom->L[il];
        if (G.nleaf == 0) continue;
        HIPCK(launch_residual_max<double>(D, G.Nb, lv64(s, il), lv64(s, il - 1), phi_zero, s->d_norm_slots,
                                          s->n_launch, st));
    }
    HIPCK(launch_norm_reduce(s->d_norm_slots, s->d_norm, mapped ? mapped : s->h_norm_dev, s->nrhs, st));
    s->norm_slots_clean = true;
    return OCTMG_OK;
}

// Before replaying a captured graph: its norm kernels assume zero slots,
// which an eager norm cut short by an error may have left otherwise.
octmg_status clean_norm_slots(octmg_state s, hipStream_t st) {
    if (!s->norm_slots_clean) HIPCK(launch_fill_u64(s->d_norm_slots, norm_slot_words(s->nrhs), 0ull, st));
    s->norm_slots_clean = true;
    return OCTMG_OK;
}

// the norms reach the host through a pinned, host-mapped buffer, written by
// the one-workgroup kernel that reduces the norm slots (cheaper than a copy
// for a few bytes); called after residual_norm_dev or mixed_defect
octmg_status read_norms(octmg_state s, double *out, hipStream_t st) {
    if (!s->h_norm) {  // no mapped buffer (octmg_solve_noalloc): copy from d_norm
        HIPCK(hipMemcpyAsync(out, s->d_norm, sizeof(double) * s->nrhs, hipMemcpyDeviceToHost, st));
        HIPCK(hipStreamSynchronize(st));
        return OCTMG_OK;
    }
    HIPCK(hipStreamSynchronize(st));
    for (int r = 0; r < s->nrhs; r++) {
        const unsigned long long v = ((volatile unsigned long long *)s->h_norm)[r];
        std::memcpy(&out[r], &v, sizeof(double));
    }
    return OCTMG_OK;
}

// The FP32 V-cycle on the correction starts from zero (every level, so the
// refinement-boundary ghosts of adaptive trees are zero too), so its first
// red half sweep on the finest level needs nothing but the FP32 right-hand
// side of each red cell: the defect kernel writes it there directly (3D
// trees whose finest level is smoothed by separate launches with at least
// one pre-smoothing step).  The same bits as the half sweep.
static bool mixed_red_preset(const octmg_state_s *s) {
    const int top = (int)s->geom->L.size() - 1;
    return s->red_preset && s->geom->tree.D == 3 && top >= 1 && s->fused_top < top && s->n_down >= 1;
}

// one outer step of the mixed-precision defect correction: FP64 defect on
// the leaves (norm into d_norm), FP32 cycle on the correction, FP64 update.
// next_v: the correction that follows is a V-cycle (mixed_red_preset applies)
octmg_status mixed_defect(octmg_state s, hipStream_t st, bool next_v, unsigned long long *mapped = nullptr) {
    const int red = next_v && mixed_red_preset(s) ? 1 : 0;
    const int top = (int)s->geom->L.size() - 1;
    Engine<double> e64{s, st};
    STCK(e64.sync_down());
    if (!s->norm_slots_clean) HIPCK(launch_fill_u64(s->d_norm_slots, norm_slot_words(s->nrhs), 0ull, st));
    s->norm_slots_clean = false;
    const int D = s->geom->tree.D;
    // The correction starts from zero.  The defect below zeroes it on every
    // leaf block, and restriction overwrites every parent block before the
    // cycle reads it, except where a refinement-boundary ghost reads a
    // coarse parent block first (adaptive trees): only there, and never on
    // the finest level (all leaves), is it cleared here.
    if (s->geom->tree.adaptive) {
        for (int il = 0; il + 1 < (int)s->geom->L.size(); il++) {
            const long long n = s->stride[il] * s->nrhs;
            HIPCK(launch_fillf(s->f32[il].phi, n, 0.0f, st));
        }
    }
    for (int il = 0; il < (int)s->geom->L.size(); il++) {
        const GeomLevel &G = s->geom->L[il];
        if (G.nleaf == 0) continue;
        HIPCK(launch_defect(D, G.Nb, lv64(s, il), lv64(s, il - 1), lv32(s, il), G.d_leaf_blocks, G.nleaf,
                            s->d_norm_slots, s->n_launch, st, il == top ? red : 0));
    }
    HIPCK(launch_norm_reduce(s->d_norm_slots, s->d_norm, mapped ? mapped : s->h_norm_dev, s->nrhs, st));
    s->norm_slots_clean = true;
    return OCTMG_OK;
}

// The FP64 update phi += e can ride on the correction's last black half
// sweep of each level with leaves (3D, with post-smoothing): those levels
// that the final V-cycle smooths by separate launches (k_gs_half3_update);
// the others take k_update.
static bool mixed_update_fused(const octmg_state_s *s) {
    return s->update_fused && s->geom->tree.D == 3 && s->n_up >= 1;
}

octmg_status mixed_correct(octmg_state s, int kind, hipStream_t st) {
    Engine<float> e32{s, st};
    e32.upd = mixed_update_fused(s);
    // only leaf values are passed on; the defect before a V-cycle has done
    // its first red half sweep
    STCK(e32.cycle(kind, kind == OCTMG_CYCLE_FMG ? 0 : 1, false, kind == OCTMG_CYCLE_V && mixed_red_preset(s)));
    const int D = s->geom->tree.D;
    for (int il = 0; il < (int)s->geom->L.size(); il++) {
        const GeomLevel &G = s->geom->L[il];
        if (G.nleaf == 0 || (il < 64 && (e32.upd_levels >> il) & 1)) continue;
        HIPCK(launch_update(D, G.Nb, lv64(s, il), lv32(s, il), G.d_leaf_blocks, G.nleaf, s->n_launch, st));
    }
    return OCTMG_OK;
}

void drop_graphs(octmg_state s) {
    for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    s->graphs.clear();
}

// (re)build the device tables of the fused bottom of the V-cycle; captured
// graphs bake in the cycle structure and are dropped
// level tables (device copies) of levels 0..top for the bottom kernels
void bottom_tables(octmg_state s, int top, SmallLevels<double> &h64, SmallLevels<float> &h32) {
    h64 = SmallLevels<double>{};
    h32 = SmallLevels<float>{};
    for (int il = 0; il <= top; il++) {
        // these kernels walk every rhs themselves (flags skip finished ones)
        h64.L[il] = lv64(s, il);
        h64.L[il].lanes = nullptr;
        h64.N[il] = s->geom->L[il].Nb;
        if (s->precision == OCTMG_MIXED) h32.L[il] = lv32(s, il);
        h32.L[il].lanes = nullptr;
        h32.N[il] = s->geom->L[il].Nb;
    }
    h64.n_down = h32.n_down = s->n_down;
    h64.n_up = h32.n_up = s->n_up;
    h64.nrhs = h32.nrhs = s->nrhs;
    h64.into_old = h32.into_old = s->geom->tree.adaptive ? 1 : 0;
    h64.M = h32.M = s->geom->d_M;
    h64.S = h32.S = s->geom->d_S;
}

octmg_status setup_fused(octmg_state s) {
    drop_graphs(s);
    s->fused_top = 0;
    if (s->fused_max_blocks <= 0 || s->geom->tree.D != 3) return OCTMG_OK;
    int ft = 0;
    for (int il = 0; il < (int)s->geom->L.size() && il < kMaxSmallLevels; il++) {
        if (s->geom->L[il].nblocks > s->fused_max_blocks) break;
        ft = il;
    }
    if (ft < 1) return OCTMG_OK;
    SmallLevels<double> h64;
    SmallLevels<float> h32;
    bottom_tables(s, ft, h64, h32);
    if (!s->d_small64) {
        HIPCK(s->pool.alloc(&s->d_small64, 1));
        HIPCK(s->pool.alloc(&s->d_small32, 1));
        HIPCK(small_vcycle_max_grid<double>(&s->fused_grid64));
        HIPCK(small_vcycle_max_grid<float>(&s->fused_grid32));
    }
    if (s->fused_grid64 < 1 || s->fused_grid32 < 1) return OCTMG_OK;
    HIPCK(hipMemcpy(s->d_small64, &h64, sizeof(h64), hipMemcpyHostToDevice));
    HIPCK(hipMemcpy(s->d_small32, &h32, sizeof(h32), hipMemcpyHostToDevice));
    s->fused_top = ft;
    return OCTMG_OK;
}

octmg_status check_level(octmg_state s, int level) {
    if (!s) return fail(OCTMG_ERR_INVALID, "null state");
    if (level < 0 || level >= (int)s->geom->L.size()) return fail(OCTMG_ERR_INVALID, "level out of range");
    return OCTMG_OK;
}

octmg_status validate_desc(const octmg_geom_desc *d) {
    if (!d) return fail(OCTMG_ERR_INVALID, "null descriptor");
    if (!(d->eps_tol > 0.0 && d->eps_tol < 0.5)) return fail(OCTMG_ERR_INVALID, "eps_tol must be in (0, 0.5)");
    if (!(d->mask_factor > 0.0)) return fail(OCTMG_ERR_INVALID, "mask_factor must be > 0");
    if (d->lsf_kind < OCTMG_LSF_NONE || d->lsf_kind > OCTMG_LSF_CALLBACK) return fail(OCTMG_ERR_INVALID, "unknown lsf_kind");
    if (d->lsf_kind == OCTMG_LSF_CALLBACK && !d->lsf_fn) return fail(OCTMG_ERR_INVALID, "lsf_fn is null");
    if (d->lsf_kind == OCTMG_LSF_SPHERES && (d->lsf_n < 1 || d->lsf_n > 100000))
        return fail(OCTMG_ERR_INVALID, "lsf_n out of range");
    if (d->lsf_kind != OCTMG_LSF_NONE && d->lsf_kind != OCTMG_LSF_CALLBACK && !d->lsf_params)
        return fail(OCTMG_ERR_INVALID, "lsf_params is null");
    if (d->neumann_faces < 0 || d->neumann_faces >= (1 << (2 * d->dim)))
        return fail(OCTMG_ERR_INVALID, "neumann_faces has bits beyond the 2D faces");
    if (d->neumann_faces == (1 << (2 * d->dim)) - 1 && d->lsf_kind == OCTMG_LSF_NONE)
        return fail(OCTMG_ERR_INVALID, "all faces zero-flux without an interface: the operator is singular");
    if (d->uniform_level < 0 || d->uniform_level > d->max_level) return fail(OCTMG_ERR_INVALID, "bad uniform_level");
    return OCTMG_OK;
}

std::vector<double> copy_params(const octmg_geom_desc &d) {
    const bool shape = d.lsf_kind >= OCTMG_LSF_SPHEROID && d.lsf_kind <= OCTMG_LSF_ASTROID;
    int np = d.lsf_kind == OCTMG_LSF_SPHERES      ? 4 * d.lsf_n
             : d.lsf_kind == OCTMG_LSF_CYLINDER_Z   ? 3
             : d.lsf_kind == OCTMG_LSF_ELECTRODES   ? 11
             : shape                                ? 5
                                                    : 0;
    std::vector<double> p(np + 1, 0.0);
    if (np && d.lsf_params) std::memcpy(p.data(), d.lsf_params, np * sizeof(double));
    return p;
}

}  // namespace

// ===================================================================== ABI
extern "C" {

const char *octmg_last_error(void) { return g_last_error.c_str(); }
int octmg_version(void) { return 1; }

octmg_status octmg_plan_levels(const octmg_geom_desc *d, int *n_levels, int64_t *info) {
    STCK(validate_desc(d));
    if (!n_levels || !info) return fail(OCTMG_ERR_INVALID, "null output");
    octmg_geom_desc dd = *d;
    std::vector<double> p = copy_params(dd);
    dd.lsf_params = p.data();
    Tree t;
    std::string err;
    if (!build_tree(dd, &t, &err)) return fail(OCTMG_ERR_INVALID, err);
    *n_levels = (int)t.lv.size();
    for (size_t il = 0; il < t.lv.size(); il++) {
        const TreeLevel &L = t.lv[il];
        int nl = 0;
        for (auto f : L.leaf) nl += f;
        info[4 * il + 0] = L.n;
        info[4 * il + 1] = L.Nb;
        info[4 * il + 2] = L.nblocks();
        info[4 * il + 3] = nl;
    }
    return OCTMG_OK;
}

octmg_status octmg_plan_blocks(const octmg_geom_desc *d, int level, int *pos, int *leaf) {
    STCK(validate_desc(d));
    octmg_geom_desc dd = *d;
    std::vector<double> p = copy_params(dd);
    dd.lsf_params = p.data();
    Tree t;
    std::string err;
    if (!build_tree(dd, &t, &err)) return fail(OCTMG_ERR_INVALID, err);
    if (level < 0 || level >= (int)t.lv.size()) return fail(OCTMG_ERR_INVALID, "level out of range");
    const TreeLevel &L = t.lv[level];
    std::memcpy(pos, L.pos.data(), L.pos.size() * sizeof(int));
    for (int b = 0; b < L.nblocks(); b++) leaf[b] = L.leaf[b];
    return OCTMG_OK;
}

// Device tables, FP64 interface setup and coarse inverse of G->tree.  With
// `reuse` (the geometry G was adapted from), the records of unchanged
// blocks are copied instead of recomputed; stats[0..3] += blocks kept,
// blocks set up, records kept, records computed.
static octmg_status setup_geometry(octmg_geom_s *G, const octmg_geom_s *reuse, int64_t *stats) {
    const int D = G->tree.D;
    const int nlev = (int)G->tree.lv.size();
    G->L.resize(nlev);

    double *d_params = nullptr;
    HIPCK(G->pool.alloc(&d_params, G->params.size()));
    HIPCK(hipMemcpy(d_params, G->params.data(), G->params.size() * sizeof(double), hipMemcpyHostToDevice));
    const int nbisect = (int)std::ceil(-std::log(G->desc.eps_tol) / std::log(2.0));
    const int ngolden = (int)std::ceil(std::log(G->desc.eps_tol) / std::log(0.5 * (std::sqrt(5.0) - 1.0)));

    // a level set given as a host function runs the setup passes on the host
    const bool host_lsf = G->desc.lsf_kind == OCTMG_LSF_CALLBACK;
    long long leaf_base = 0, pt_base = 0;
    bool coarse_kept = false;  // level 0 unchanged: the coarse inverse carries over
    for (int il = 0; il < nlev; il++) {
        const TreeLevel &T = G->tree.lv[il];
        GeomLevel &L = G->L[il];
        L.n = T.n;
        L.Nb = T.Nb;
        L.nb = T.nb;
        L.nblocks = T.nblocks();
        L.cpb = cells_per_block(D, T.Nb);
        L.nface = D == 3 ? T.n * T.n : T.n;
        L.dx = 1.0 / (double)T.n;
        std::vector<int4> pos4(L.nblocks);
        std::vector<int> leaf(L.nblocks);
        for (int b = 0; b < L.nblocks; b++) {
            pos4[b] = make_int4(T.pos[3 * b], T.pos[3 * b + 1], T.pos[3 * b + 2], 0);
            leaf[b] = T.leaf[b];
            if (T.leaf[b]) L.leaf_blocks.push_back(b);
        }
        L.nleaf = (int)L.leaf_blocks.size();
        L.leaf_base = leaf_base;
        leaf_base += (long long)L.nleaf * L.cpb;
        HIPCK(G->pool.alloc(&L.d_pos, L.nblocks));
        HIPCK(G->pool.alloc(&L.d_lut, T.lut.size()));
        HIPCK(G->pool.alloc(&L.d_leaf, L.nblocks));
        HIPCK(G->pool.alloc(&L.d_map_off, L.nblocks));
        HIPCK(G->pool.alloc(&L.d_leaf_blocks, std::max(1, L.nleaf)));
        HIPCK(hipMemcpy(L.d_pos, pos4.data(), L.nblocks * sizeof(int4), hipMemcpyHostToDevice));
        {
            // face neighbour table: one lookup per block instead of a
            // position load followed by six table lookups in every kernel
            std::vector<int> nbr((size_t)8 * L.nblocks, -2);
            for (int b = 0; b < L.nblocks; b++)
                for (int f = 0; f < 2 * D; f++) {
                    int q[3] = {pos4[b].x, pos4[b].y, pos4[b].z};
                    q[f >> 1] += (f & 1) ? 1 : -1;
                    bool in = true;
                    for (int a = 0; a < D; a++) in = in && q[a] >= 0 && q[a] < L.nb;
                    if (!in) continue;
                    const long long li = D == 3 ? ((long long)q[2] * L.nb + q[1]) * L.nb + q[0]
                                                : (long long)q[1] * L.nb + q[0];
                    nbr[(size_t)8 * b + f] = T.lut[li];
                }
            HIPCK(G->pool.alloc(&L.d_nbr, (size_t)2 * L.nblocks));
            HIPCK(hipMemcpy(L.d_nbr, nbr.data(), nbr.size() * sizeof(int), hipMemcpyHostToDevice));
        }
        HIPCK(hipMemcpy(L.d_lut, T.lut.data(), T.lut.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCK(hipMemcpy(L.d_leaf, leaf.data(), L.nblocks * sizeof(int), hipMemcpyHostToDevice));
        if (L.nleaf)
            HIPCK(hipMemcpy(L.d_leaf_blocks, L.leaf_blocks.data(), L.nleaf * sizeof(int), hipMemcpyHostToDevice));

        // ---- FP64 interface setup of this level (two passes)
        SetupLevel S{};
        S.D = D;
        S.n = L.n;
        S.Nb = L.Nb;
        S.nblocks = L.nblocks;
        S.nb = L.nb;
        S.dx = L.dx;
        for (int a = 0; a < 3; a++) S.lo[a] = G->desc.lo[a];
        S.pos = L.d_pos;
        S.lut = L.d_lut;
        S.leaf = L.d_leaf;
        S.lsf_kind = G->desc.lsf_kind;
        S.lsf_n = G->desc.lsf_n;
        S.lsf_params = d_params;
        S.lsf_fn = G->desc.lsf_fn;
        S.lsf_user = G->desc.lsf_user;
        S.mask_L = G->desc.mask_factor * std::sqrt((double)D) * L.dx;
        S.w_min = G->desc.w_min;
        S.nbisect = nbisect;
        S.ngolden = ngolden;
        // blocks of the previous geometry with the same level, position and
        // leaf status keep their records; only the others are set up
        const GeomLevel *Lo = reuse && il < (int)reuse->L.size() ? &reuse->L[il] : nullptr;
        const TreeLevel *To = reuse && il < (int)reuse->tree.lv.size() ? &reuse->tree.lv[il] : nullptr;
        std::vector<int> old_of(L.nblocks, -1), fresh;
        for (int b = 0; b < L.nblocks; b++) {
            if (To && To->nb == T.nb) {
                const long long li = D == 3 ? ((long long)pos4[b].z * T.nb + pos4[b].y) * T.nb + pos4[b].x
                                            : (long long)pos4[b].y * T.nb + pos4[b].x;
                const int ob = To->lut[li];
                if (ob >= 0 && To->leaf[ob] == T.leaf[b]) old_of[b] = ob;
            }
            if (old_of[b] < 0) fresh.push_back(b);
        }
        if (stats) {
            stats[0] += L.nblocks - (long long)fresh.size();
            stats[1] += (long long)fresh.size();
        }
        if (il == 0) coarse_kept = reuse && fresh.empty();
        DevPool tmp(G->allocator(), G->device);  // this level's temporaries
        int *d_counts = nullptr, *d_fresh = nullptr;
        unsigned char *d_flags = nullptr;  // per cell: custom-cell flag of the count pass
        HIPCK(tmp.alloc(&d_counts, (size_t)2 * L.nblocks));
        HIPCK(tmp.alloc(&d_fresh, std::max<size_t>(1, fresh.size())));
        std::vector<int> counts(2 * L.nblocks, 0);
        SetupLevel H{};  // host view of S for a host level set
        if (!fresh.empty()) {
            HIPCK(hipMemcpy(d_fresh, fresh.data(), sizeof(int) * fresh.size(), hipMemcpyHostToDevice));
            S.blocks = (int)fresh.size() == L.nblocks ? nullptr : d_fresh;
            S.nlist = (int)fresh.size();
            if (host_lsf) {
                H = S;
                H.pos = pos4.data();
                H.lut = T.lut.data();
                H.leaf = leaf.data();
                H.lsf_params = G->params.data();
                H.blocks = S.blocks ? fresh.data() : nullptr;
                host_setup_count(H, counts.data());
            } else {
                HIPCK(tmp.alloc(&d_flags, (size_t)L.nblocks * L.cpb));
                HIPCK(hipMemset(d_counts, 0, sizeof(int) * 2 * L.nblocks));
                HIPCK(launch_setup_count(S, d_counts, d_flags, nullptr));
                HIPCK(hipMemcpy(counts.data(), d_counts, sizeof(int) * 2 * L.nblocks, hipMemcpyDeviceToHost));
            }
        }
        for (int b = 0; b < L.nblocks; b++)
            if (old_of[b] >= 0) {
                counts[2 * b] = Lo->h_nrec[old_of[b]];
                counts[2 * b + 1] = Lo->h_npt[old_of[b]];
            }
        std::vector<int> rec_off(L.nblocks), pt_off(L.nblocks), map_off(L.nblocks, -1);
        int nrec = 0, nib = 0;
        long long npt = 0;
        for (int b = 0; b < L.nblocks; b++) {
            rec_off[b] = nrec;
            pt_off[b] = (int)npt;
            if (counts[2 * b] > 0) map_off[b] = (nib++) * L.cpb;
            nrec += counts[2 * b];
            npt += counts[2 * b + 1];
        }
        L.h_nrec.resize(L.nblocks);
        L.h_npt.resize(L.nblocks);
        for (int b = 0; b < L.nblocks; b++) {
            L.h_nrec[b] = counts[2 * b];
            L.h_npt[b] = counts[2 * b + 1];
        }
        L.h_rec_off = rec_off;
        L.h_pt_off = pt_off;
        L.h_map_off = map_off;
        L.nrec = nrec;
        L.npts = npt;
        L.n_iface_blocks = nib;
        L.pt_base = pt_base;
        pt_base += npt;
        HIPCK(hipMemcpy(L.d_map_off, map_off.data(), sizeof(int) * L.nblocks, hipMemcpyHostToDevice));
        if (nrec) {
            int *d_roff = nullptr, *d_poff = nullptr;
            HIPCK(tmp.alloc(&d_roff, (size_t)L.nblocks));
            HIPCK(tmp.alloc(&d_poff, (size_t)L.nblocks));
            HIPCK(hipMemcpy(d_roff, rec_off.data(), sizeof(int) * L.nblocks, hipMemcpyHostToDevice));
            HIPCK(hipMemcpy(d_poff, pt_off.data(), sizeof(int) * L.nblocks, hipMemcpyHostToDevice));
            HIPCK(G->pool.alloc(&L.d_map, (size_t)nib * L.cpb));
            HIPCK(hipMemset(L.d_map, 0xFF, sizeof(int) * (size_t)nib * L.cpb));
            HIPCK(G->pool.alloc(&L.d_meta, (size_t)4 * nrec));
            HIPCK(G->pool.alloc(&L.d_d6, (size_t)6 * nrec));
            HIPCK(G->pool.alloc(&L.d_cfull, (size_t)6 * nrec));
            HIPCK(G->pool.alloc(&L.d_rec8, (size_t)8 * nrec));
            HIPCK(G->pool.alloc(&L.d_rec8f, (size_t)8 * nrec));
            HIPCK(G->pool.alloc(&L.d_pts, (size_t)3 * std::max<long long>(1, npt)));
            HIPCK(G->pool.alloc(&L.d_inside, (size_t)nrec));
            if (!fresh.empty() && host_lsf) {
                // records of the fresh blocks on the host, uploaded whole; the
                // kept blocks' entries are filled in by the copy below
                std::vector<int> map((size_t)nib * L.cpb, -1), meta((size_t)4 * nrec, 0), inside(nrec, 0);
                std::vector<double> d6((size_t)6 * nrec, 0.0), cfull((size_t)6 * nrec, 0.0), rec8((size_t)8 * nrec, 0.0);
                std::vector<float> rec8f((size_t)8 * nrec, 0.0f);
                std::vector<double> pts((size_t)3 * std::max<long long>(1, npt), 0.0);
                host_setup_emit(H, rec_off.data(), pt_off.data(), map_off.data(), map.data(), meta.data(), d6.data(),
                                cfull.data(), rec8.data(), rec8f.data(), pts.data(), inside.data());
                HIPCK(hipMemcpy(L.d_map, map.data(), sizeof(int) * map.size(), hipMemcpyHostToDevice));
                HIPCK(hipMemcpy(L.d_meta, meta.data(), sizeof(int) * meta.size(), hipMemcpyHostToDevice));
                HIPCK(hipMemcpy(L.d_inside, inside.data(), sizeof(int) * inside.size(), hipMemcpyHostToDevice));
                HIPCK(hipMemcpy(L.d_d6, d6.data(), sizeof(double) * d6.size(), hipMemcpyHostToDevice));
                HIPCK(hipMemcpy(L.d_cfull, cfull.data(), sizeof(double) * cfull.size(), hipMemcpyHostToDevice));
                HIPCK(hipMemcpy(L.d_rec8, rec8.data(), sizeof(double) * rec8.size(), hipMemcpyHostToDevice));
                HIPCK(hipMemcpy(L.d_rec8f, rec8f.data(), sizeof(float) * rec8f.size(), hipMemcpyHostToDevice));
                HIPCK(hipMemcpy(L.d_pts, pts.data(), sizeof(double) * pts.size(), hipMemcpyHostToDevice));
            } else if (!fresh.empty()) {
                HIPCK(launch_setup_emit(S, d_flags, d_roff, d_poff, L.d_map_off, L.d_map, L.d_meta, L.d_d6, L.d_cfull,
                                        L.d_rec8, L.d_rec8f, L.d_pts, L.d_inside, nullptr));
            }
            std::vector<ReuseBlock> keep;
            for (int b = 0; b < L.nblocks; b++) {
                const int ob = old_of[b];
                if (ob < 0 || (counts[2 * b] == 0 && map_off[b] < 0)) continue;
                keep.push_back({ob, b, Lo->h_rec_off[ob], rec_off[b], counts[2 * b], Lo->h_pt_off[ob], pt_off[b],
                                counts[2 * b + 1], Lo->h_map_off[ob], map_off[b]});
            }
            if (stats)
                for (const ReuseBlock &k : keep) stats[2] += k.nrec;
            if (!keep.empty()) {
                ReuseBlock *d_keep = nullptr;
                HIPCK(tmp.alloc(&d_keep, keep.size()));
                HIPCK(hipMemcpy(d_keep, keep.data(), sizeof(ReuseBlock) * keep.size(), hipMemcpyHostToDevice));
                const ReuseArrays ra{Lo->d_map, Lo->d_meta, Lo->d_inside, Lo->d_d6, Lo->d_cfull, Lo->d_rec8,
                                     Lo->d_pts, Lo->d_rec8f};
                const ReuseArrays rb{L.d_map, L.d_meta, L.d_inside, L.d_d6, L.d_cfull, L.d_rec8, L.d_pts, L.d_rec8f};
                HIPCK(launch_reuse_records(d_keep, (int)keep.size(), L.cpb, ra, rb, nullptr));
            }
            HIPCK(hipDeviceSynchronize());
        }
        G->n_rec += nrec;
        G->n_iface_blocks += nib;
        G->n_dom += 2LL * D * L.nface;
    }
    G->n_leaf = leaf_base;
    G->n_pts = pt_base;

    // ---- coarsest grid: dense operator and row-equilibrated inverse
    {
        const GeomLevel &L0 = G->L[0];
        if (L0.nblocks != 1 || L0.Nb != 8) return fail(OCTMG_ERR_GEOMETRY, "coarsest level must be one 8^D block");
        const int n0 = L0.cpb;
        DevPool tmp(G->allocator(), G->device);
        double *d_A = nullptr, *d_mult = nullptr;
        int *d_fail = nullptr;
        HIPCK(tmp.alloc(&d_A, (size_t)n0 * n0));
        HIPCK(tmp.alloc(&d_mult, (size_t)n0));
        HIPCK(tmp.alloc(&d_fail, 1));
        HIPCK(hipMemset(d_fail, 0, sizeof(int)));
        HIPCK(G->pool.alloc(&G->d_M, (size_t)n0 * n0));
        HIPCK(G->pool.alloc(&G->d_S, (size_t)n0));
        if (coarse_kept) {
            HIPCK(hipMemcpy(G->d_M, reuse->d_M, sizeof(double) * n0 * n0, hipMemcpyDeviceToDevice));
            HIPCK(hipMemcpy(G->d_S, reuse->d_S, sizeof(double) * n0, hipMemcpyDeviceToDevice));
        } else {
            int mo = -1;
            HIPCK(hipMemcpy(&mo, L0.d_map_off, sizeof(int), hipMemcpyDeviceToHost));
            HIPCK(launch_coarse_assemble(D, L0.Nb, L0.dx, mo >= 0 ? L0.d_map + mo : nullptr, L0.d_rec8,
                                         G->desc.neumann_faces, d_A, nullptr));
            HIPCK(launch_gauss_jordan(n0, d_A, G->d_M, G->d_S, d_mult, d_fail, nullptr));
            int hf = 0;
            HIPCK(hipMemcpy(&hf, d_fail, sizeof(int), hipMemcpyDeviceToHost));
            if (hf) return fail(OCTMG_ERR_GEOMETRY, "coarse-grid operator is singular");
        }
    }
    if (stats) stats[3] += G->n_rec;
    HIPCK(hipDeviceSynchronize());
    return OCTMG_OK;
}

static octmg_status check_device(int hip_device) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(OCTMG_ERR_HIP, "no HIP device");
    if (hip_device < 0 || hip_device >= ndev) return fail(OCTMG_ERR_INVALID, "bad device index");
    return OCTMG_OK;
}

octmg_status octmg_ctx_create(int hip_device, const octmg_allocator *alloc, const char *tune_cache_path,
                              octmg_ctx *out) {
    if (!out) return fail(OCTMG_ERR_INVALID, "null output");
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(OCTMG_ERR_INVALID, "allocator needs alloc and free");
    STCK(check_device(hip_device));
    octmg_ctx c = new octmg_ctx_s();
    c->device = hip_device;
    if (alloc) {
        c->alloc = *alloc;
        c->has_alloc = true;
    }
    if (tune_cache_path) c->tune_path = tune_cache_path;
    *out = c;
    return OCTMG_OK;
}

void octmg_ctx_destroy(octmg_ctx c) { release_ctx(c); }

octmg_status octmg_geom_create(const octmg_geom_desc *d, int hip_device, octmg_geom *out) {
    return octmg_geom_create_in(nullptr, d, hip_device, out);
}

octmg_status octmg_geom_create_in(octmg_ctx ctx, const octmg_geom_desc *d, int hip_device, octmg_geom *out) {
    STCK(validate_desc(d));
    if (!out) return fail(OCTMG_ERR_INVALID, "null output");
    *out = nullptr;
    if (ctx) hip_device = ctx->device;
    STCK(check_device(hip_device));
    HIPCK(hipSetDevice(hip_device));
    std::unique_ptr<octmg_geom_s> G(new octmg_geom_s());
    if (ctx) {
        G->ctx = ctx;  // referenced once the geometry exists (below)
        G->pool.a = ctx->allocator();
    }
    G->pool.device = hip_device;
    G->desc = *d;
    G->params = copy_params(*d);
    G->desc.lsf_params = G->params.data();
    G->device = hip_device;
    std::string err;
    if (!build_tree(G->desc, &G->tree, &err)) return fail(OCTMG_ERR_INVALID, err);
    STCK(setup_geometry(G.get(), nullptr, nullptr));
    if (G->ctx) G->ctx->refs++;
    *out = G.release();
    return OCTMG_OK;
}

octmg_status octmg_geom_adapt(octmg_geom g, const int8_t *flags, int reuse, octmg_geom *out, int64_t *stats) {
    if (!g || !flags || !out) return fail(OCTMG_ERR_INVALID, "null argument");
    *out = nullptr;
    HIPCK(hipSetDevice(g->device));
    std::unique_ptr<octmg_geom_s> G(new octmg_geom_s());
    if (g->ctx) {
        G->ctx = g->ctx;
        G->pool.a = g->ctx->allocator();
    }
    G->pool.device = g->device;
    G->desc = g->desc;
    G->params = g->params;
    G->desc.lsf_params = G->params.data();
    G->device = g->device;
    std::string err;
    if (!adapt_tree(G->desc, g->tree, flags, &G->tree, &err)) return fail(OCTMG_ERR_INVALID, err);
    if (stats) std::memset(stats, 0, 4 * sizeof(int64_t));
    STCK(setup_geometry(G.get(), reuse ? g : nullptr, stats));
    if (stats) stats[3] -= stats[2];
    if (G->ctx) G->ctx->refs++;
    *out = G.release();
    return OCTMG_OK;
}

void octmg_geom_destroy(octmg_geom g) { release_geom(g); }

octmg_status octmg_geom_info(octmg_geom g, int64_t *info) {
    if (!g || !info) return fail(OCTMG_ERR_INVALID, "null argument");
    long long blocks = 0;
    for (auto &L : g->L) blocks += L.nblocks;
    info[0] = (int64_t)g->L.size();
    info[1] = g->n_leaf;
    info[2] = g->n_pts;
    info[3] = g->n_dom;
    info[4] = g->n_rec;
    info[5] = (int64_t)g->pool.bytes;
    info[6] = blocks;
    info[7] = g->n_iface_blocks;
    return OCTMG_OK;
}

octmg_status octmg_geom_level_info(octmg_geom g, int level, int64_t *out) {
    if (!g || !out) return fail(OCTMG_ERR_INVALID, "null argument");
    if (level < 0 || level >= (int)g->L.size()) return fail(OCTMG_ERR_INVALID, "level out of range");
    const GeomLevel &L = g->L[level];
    out[0] = L.n;
    out[1] = L.Nb;
    out[2] = L.nblocks;
    out[3] = L.nleaf;
    out[4] = L.nrec;
    out[5] = L.npts;
    out[6] = L.nface;
    out[7] = L.n_iface_blocks;
    return OCTMG_OK;
}

octmg_status octmg_geom_leaf_coords(octmg_geom g, double *xyz, int *level) {
    if (!g) return fail(OCTMG_ERR_INVALID, "null geometry");
    const int D = g->tree.D;
    long long n = 0;
    for (size_t il = 0; il < g->L.size(); il++) {
        const GeomLevel &L = g->L[il];
        const TreeLevel &T = g->tree.lv[il];
        for (int b : L.leaf_blocks)
            for (int c = 0; c < L.cpb; c++, n++) {
                const int l[3] = {c % L.Nb, (c / L.Nb) % L.Nb, D == 3 ? c / (L.Nb * L.Nb) : 0};
                for (int a = 0; a < 3; a++) {
                    double v = 0.0;
                    if (a < D) v = g->desc.lo[a] + ((double)(T.pos[3 * b + a] * L.Nb + l[a]) + 0.5) * L.dx;
                    if (xyz) xyz[3 * n + a] = v;
                }
                if (level) level[n] = (int)il;
            }
    }
    return OCTMG_OK;
}

octmg_status octmg_geom_iface_points(octmg_geom g, double *xyz) {
    if (!g || !xyz) return fail(OCTMG_ERR_INVALID, "null argument");
    HIPCK(hipSetDevice(g->device));
    for (auto &L : g->L)
        if (L.npts) HIPCK(hipMemcpy(xyz + 3 * L.pt_base, L.d_pts, sizeof(double) * 3 * L.npts, hipMemcpyDeviceToHost));
    return OCTMG_OK;
}

octmg_status octmg_geom_domain_points(octmg_geom g, double *xyz) {
    if (!g || !xyz) return fail(OCTMG_ERR_INVALID, "null argument");
    const int D = g->tree.D;
    long long n = 0;
    for (auto &L : g->L)
        for (int f = 0; f < 2 * D; f++) {
            const int ax = f / 2;
            for (int t = 0; t < L.nface; t++, n++) {
                const int tg[2] = {t % L.n, t / L.n};
                int m = 0;
                for (int a = 0; a < 3; a++) {
                    double v = 0.0;
                    if (a < D) {
                        if (a == ax) v = (f & 1) ? g->desc.lo[a] + 1.0 : g->desc.lo[a];
                        else v = g->desc.lo[a] + ((double)tg[m++] + 0.5) * L.dx;
                    }
                    xyz[3 * n + a] = v;
                }
            }
        }
    return OCTMG_OK;
}

octmg_status octmg_geom_records(octmg_geom g, int level, int *ids, double *d, double *coef) {
    if (!g || level < 0 || level >= (int)g->L.size()) return fail(OCTMG_ERR_INVALID, "bad argument");
    HIPCK(hipSetDevice(g->device));
    const GeomLevel &L = g->L[level];
    if (!L.nrec) return OCTMG_OK;
    const int D = g->tree.D;
    std::vector<int> meta(4 * L.nrec);
    std::vector<double> d6(6 * L.nrec), cf(6 * L.nrec), r8(8 * L.nrec);
    HIPCK(hipMemcpy(meta.data(), L.d_meta, sizeof(int) * meta.size(), hipMemcpyDeviceToHost));
    HIPCK(hipMemcpy(d6.data(), L.d_d6, sizeof(double) * d6.size(), hipMemcpyDeviceToHost));
    HIPCK(hipMemcpy(cf.data(), L.d_cfull, sizeof(double) * cf.size(), hipMemcpyDeviceToHost));
    HIPCK(hipMemcpy(r8.data(), L.d_rec8, sizeof(double) * r8.size(), hipMemcpyDeviceToHost));
    const int N = L.Nb, half = L.cpb / 2, nh = N / 2;
    for (int r = 0; r < L.nrec; r++) {
        // split index -> canonical local index
        const int si = meta[4 * r + 1], col = si / half, q = si % half;
        const int h = q % nh, j = (q / nh) % N, k = D == 3 ? q / (nh * N) : 0;
        const int i = 2 * h + ((col + j + k) & 1);
        if (ids) {
            ids[3 * r] = meta[4 * r];
            ids[3 * r + 1] = D == 3 ? (k * N + j) * N + i : j * N + i;
            ids[3 * r + 2] = meta[4 * r + 2];
        }
        for (int kk = 0; kk < 6; kk++) {
            if (d) d[6 * r + kk] = d6[6 * r + kk];
            if (coef) coef[8 * r + kk] = cf[6 * r + kk];
        }
        if (coef) {
            coef[8 * r + 6] = r8[8 * r + 6];
            coef[8 * r + 7] = 0.0;
        }
    }
    return OCTMG_OK;
}

octmg_status octmg_geom_block_positions(octmg_geom g, int level, int *pos, int *leaf) {
    if (!g || level < 0 || level >= (int)g->L.size()) return fail(OCTMG_ERR_INVALID, "bad argument");
    const TreeLevel &T = g->tree.lv[level];
    if (pos) std::memcpy(pos, T.pos.data(), T.pos.size() * sizeof(int));
    if (leaf)
        for (int b = 0; b < T.nblocks(); b++) leaf[b] = T.leaf[b];
    return OCTMG_OK;
}

octmg_status octmg_state_create(octmg_geom g, int n_rhs, int precision, octmg_state *out) {
    if (!g || !out) return fail(OCTMG_ERR_INVALID, "null argument");
    if (n_rhs < 1 || n_rhs > 4096) return fail(OCTMG_ERR_INVALID, "n_rhs out of range");
    if (precision != OCTMG_FP64 && precision != OCTMG_MIXED) return fail(OCTMG_ERR_INVALID, "bad precision");
    HIPCK(hipSetDevice(g->device));
    std::unique_ptr<octmg_state_s> s(new octmg_state_s());
    s->geom = g;
    s->pool.a = g->allocator();
    s->pool.device = g->device;
    s->nrhs = n_rhs;
    s->precision = precision;
    const int nlev = (int)g->L.size(), D = g->tree.D;
    s->f64.resize(nlev);
    s->f32.resize(nlev);
    s->stride.resize(nlev);
    for (int il = 0; il < nlev; il++) {
        const GeomLevel &L = g->L[il];
        const long long cells = (long long)L.nblocks * L.cpb;
        s->stride[il] = cells;
        const size_t n = (size_t)cells * n_rhs;
        Fields64 &F = s->f64[il];
        HIPCK(s->pool.alloc(&F.phi, n));
        HIPCK(s->pool.alloc(&F.g, n));
        HIPCK(s->pool.alloc(&F.old, n));
        if (D == 3) HIPCK(s->pool.alloc(&F.bp, n));
        HIPCK(s->pool.alloc(&F.b, std::max(1, L.nrec)));
        HIPCK(s->pool.alloc(&F.bcv, (size_t)2 * D * L.nface));
        HIPCK(s->pool.alloc(&F.pb, (size_t)std::max<long long>(1, L.npts)));
        HIPCK(launch_fill(F.pb, std::max<long long>(1, L.npts), 0.0, nullptr));
        HIPCK(launch_fill(F.phi, n, 0.0, nullptr));
        HIPCK(launch_fill(F.g, n, 0.0, nullptr));
        HIPCK(launch_fill(F.old, n, 0.0, nullptr));
        HIPCK(launch_fill(F.b, std::max(1, L.nrec), 0.0, nullptr));
        HIPCK(launch_fill(F.bcv, (long long)2 * D * L.nface, 0.0, nullptr));
        if (precision == OCTMG_MIXED) {
            Fields32 &H = s->f32[il];
            HIPCK(s->pool.alloc(&H.phi, n));
            HIPCK(s->pool.alloc(&H.g, n));
            HIPCK(s->pool.alloc(&H.old, n));
            if (D == 3) HIPCK(s->pool.alloc(&H.bp, n));
            HIPCK(launch_fillf(H.phi, n, 0.0f, nullptr));
            HIPCK(launch_fillf(H.g, n, 0.0f, nullptr));
            HIPCK(launch_fillf(H.old, n, 0.0f, nullptr));
        }
    }
    HIPCK(s->pool.alloc(&s->d_norm, n_rhs));
    HIPCK(s->pool.alloc(&s->d_norm_slots, (size_t)norm_slot_words(n_rhs)));
    HIPCK(s->pool.alloc(&s->d_flag, 1));
    HIPCK(s->pool.alloc(&s->d_active, 2 * (size_t)n_rhs));
    s->active_host.assign(n_rhs, 1);
    s->n_launch = n_rhs;
    for (int r = 0; r < n_rhs; r++) s->lanes_host.push_back(r);
    {
        std::vector<int> ctrl(s->active_host);
        ctrl.insert(ctrl.end(), s->lanes_host.begin(), s->lanes_host.end());
        HIPCK(hipMemcpy(s->d_active, ctrl.data(), sizeof(int) * ctrl.size(), hipMemcpyHostToDevice));
    }
    HIPCK(hipHostMalloc((void **)&s->h_norm, sizeof(unsigned long long) * n_rhs, hipHostMallocMapped));
    HIPCK(hipHostGetDevicePointer((void **)&s->h_norm_dev, s->h_norm, 0));
    HIPCK(s->pool.alloc(&s->d_thresh, n_rhs));
    HIPCK(s->pool.alloc(&s->d_hist, (size_t)64 * n_rhs));
    HIPCK(s->pool.alloc(&s->d_cbase, 1));
    STCK(setup_fused(s.get()));
    // the fills ran on the legacy default stream; other streams' work (a
    // server's running batches) need not be waited for
    HIPCK(hipStreamSynchronize(nullptr));
    g->refs++;
    *out = s.release();
    return OCTMG_OK;
}

void octmg_state_destroy(octmg_state s) {
    if (!s) return;
    (void)hipSetDevice(s->geom->device);
    (void)hipDeviceSynchronize();
    octmg_geom g = s->geom;
    if (s->h_norm) (void)hipHostFree(s->h_norm);
    if (s->h_ctrl) (void)hipHostFree(s->h_ctrl);
    if (s->h_begin) (void)hipHostFree(s->h_begin);
    for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
    delete s->prof;
    delete s;
    release_geom(g);
}

octmg_status octmg_profile_enable(octmg_state s, int enable) {
    if (!s) return fail(OCTMG_ERR_INVALID, "null state");
    if (!s->prof) s->prof = new Profile();
    s->prof->on = enable != 0;
    return OCTMG_OK;
}

octmg_status octmg_profile_read(octmg_state s, double *out) {
    if (!s || !out) return fail(OCTMG_ERR_INVALID, "null argument");
    HIPCK(hipSetDevice(s->geom->device));
    Profile *P = s->prof;
    double ms_total = 0.0, n = 0.0, upd = 0.0;
    if (P) {
        for (size_t i = 0; i < P->pending.size(); i++) {
            auto &pr = P->pending[i];
            HIPCK(hipEventSynchronize(pr.second));
            float ms = 0.0f;
            HIPCK(hipEventElapsedTime(&ms, pr.first, pr.second));
            ms_total += ms;
            n += P->launches[i];
            P->spare.push_back(pr.first);
            P->spare.push_back(pr.second);
        }
        P->pending.clear();
        P->launches.clear();
        upd = P->updates;
        P->updates = 0.0;
    }
    const GeomLevel &top = s->geom->L.back();
    out[0] = n;
    out[1] = ms_total;
    out[2] = upd;
    out[3] = (double)top.nblocks * top.cpb;
    return OCTMG_OK;
}

octmg_status octmg_state_set_smoothing(octmg_state s, int n_down, int n_up) {
    if (!s || n_down < 0 || n_up < 0 || n_down > 16 || n_up > 16) return fail(OCTMG_ERR_INVALID, "bad argument");
    s->n_down = n_down;
    s->n_up = n_up;
    HIPCK(hipSetDevice(s->geom->device));
    return setup_fused(s);
}

octmg_status octmg_state_set_fused_levels(octmg_state s, int max_blocks) {
    if (!s || max_blocks < 0) return fail(OCTMG_ERR_INVALID, "bad argument");
    s->fused_max_blocks = max_blocks;
    HIPCK(hipSetDevice(s->geom->device));
    return setup_fused(s);
}

octmg_status octmg_state_set_launch(octmg_state s, const octmg_launch_config *c) {
    if (!s || !c) return fail(OCTMG_ERR_INVALID, "null argument");
    if (c->block_order < 0 || c->block_order > 2 || c->bottom_max_blocks < 0 || c->graph_mode < 0 ||
        c->graph_mode > 2 || (c->bottom_kind != 0 && c->bottom_kind != 1) || c->pair_max_blocks < 0)
        return fail(OCTMG_ERR_INVALID, "bad launch configuration");
    if (c->bottom_kind == 1 && c->graph_mode != 0)
        return fail(OCTMG_ERR_INVALID, "the cooperative bottom launch cannot be captured");
    if ((c->prolong_fused != 0 && c->prolong_fused != 1) || (c->red_preset != 0 && c->red_preset != 1) ||
        (c->update_fused != 0 && c->update_fused != 1))
        return fail(OCTMG_ERR_INVALID, "bad launch configuration");
    s->block_order = c->block_order;
    s->pair_max_blocks = c->pair_max_blocks;
    s->prolong_fused = c->prolong_fused;
    s->red_preset = c->red_preset;
    s->update_fused = c->update_fused;
    s->tuned_graph = c->graph_mode;
    s->fused_max_blocks = c->bottom_kind ? c->bottom_max_blocks : 0;
    HIPCK(hipSetDevice(s->geom->device));
    return setup_fused(s);  // rebuilds the level tables and drops captured graphs
}

octmg_status octmg_state_get_launch(octmg_state s, octmg_launch_config *c) {
    if (!s || !c) return fail(OCTMG_ERR_INVALID, "null argument");
    c->block_order = s->block_order;
    c->bottom_kind = s->fused_max_blocks > 0 ? 1 : 0;
    c->bottom_max_blocks = s->fused_max_blocks;
    c->graph_mode = s->tuned_graph;
    c->pair_max_blocks = s->pair_max_blocks;
    c->prolong_fused = s->prolong_fused;
    c->red_preset = s->red_preset;
    c->update_fused = s->update_fused;
    return OCTMG_OK;
}

static octmg_status stage_in(const double *src, size_t n, int on_device, hipStream_t st, double **dev,
                             DevPool *tmp) {
    if (on_device) {
        *dev = (double *)src;
        return OCTMG_OK;
    }
    HIPCK(tmp->alloc(dev, n));
    HIPCK(hipMemcpyAsync(*dev, src, n * sizeof(double), hipMemcpyHostToDevice, st));
    return OCTMG_OK;
}

static octmg_status check_finite(octmg_state s, const double *dptr, long long n, hipStream_t st) {
    HIPCK(hipMemsetAsync(s->d_flag, 0, sizeof(int), st));
    HIPCK(launch_check_finite(dptr, n, s->d_flag, st));
    int h = 0;
    HIPCK(hipMemcpyAsync(&h, s->d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    if (h) return fail(OCTMG_ERR_NONFINITE, "input holds NaN or Inf");
    return OCTMG_OK;
}

octmg_status octmg_set_boundary(octmg_state s, const double *iface_vals, const double *domain_vals, int on_device,
                                void *stream) {
    if (!s) return fail(OCTMG_ERR_INVALID, "null state");
    s->r0_dirty = true;
    hipStream_t st = (hipStream_t)stream;
    octmg_geom g = s->geom;
    HIPCK(hipSetDevice(g->device));
    const int D = g->tree.D;
    DevPool tmp(s->geom->allocator(), s->geom->device);
    double *dv_iface = nullptr, *dv_dom = nullptr;
    if (iface_vals && g->n_pts) {
        STCK(stage_in(iface_vals, g->n_pts, on_device, st, &dv_iface, &tmp));
        STCK(check_finite(s, dv_iface, g->n_pts, st));
    }
    if (domain_vals) {
        STCK(stage_in(domain_vals, g->n_dom, on_device, st, &dv_dom, &tmp));
        STCK(check_finite(s, dv_dom, g->n_dom, st));
    }
    long long dom_off = 0;
    for (size_t il = 0; il < g->L.size(); il++) {
        const GeomLevel &L = g->L[il];
        Fields64 &F = s->f64[il];
        HIPCK(launch_boundary_terms(D, L.d_meta, L.d_cfull, L.nrec, dv_iface ? dv_iface + L.pt_base : nullptr, F.b,
                                    nullptr, st));
        if (L.npts) {
            if (dv_iface) HIPCK(hipMemcpyAsync(F.pb, dv_iface + L.pt_base, L.npts * sizeof(double), hipMemcpyDeviceToDevice, st));
            else HIPCK(launch_fill(F.pb, L.npts, 0.0, st));
        }
        const long long nf = 2LL * D * L.nface;
        if (dv_dom) HIPCK(hipMemcpyAsync(F.bcv, dv_dom + dom_off, nf * sizeof(double), hipMemcpyDeviceToDevice, st));
        else HIPCK(launch_fill(F.bcv, nf, 0.0, st));
        dom_off += nf;
    }
    HIPCK(hipStreamSynchronize(st));
    return OCTMG_OK;
}

// FP64 device copy of n caller values of type dtype (host or device)
static octmg_status stage_in_typed(const void *src, int dtype, size_t n, int on_device, hipStream_t st, double **dev,
                                   DevPool *tmp) {
    if (dtype == OCTMG_DTYPE_F64) return stage_in((const double *)src, n, on_device, st, dev, tmp);
    const float *f = (const float *)src;
    if (!on_device) {
        float *df = nullptr;
        HIPCK(tmp->alloc(&df, n));
        HIPCK(hipMemcpyAsync(df, src, n * sizeof(float), hipMemcpyHostToDevice, st));
        f = df;
    }
    HIPCK(tmp->alloc(dev, n));
    HIPCK(launch_copy_f2d(f, *dev, (long long)n, st));
    return OCTMG_OK;
}

static octmg_status check_dtype(int dtype) {
    if (dtype != OCTMG_DTYPE_F64 && dtype != OCTMG_DTYPE_F32) return fail(OCTMG_ERR_INVALID, "unknown dtype");
    return OCTMG_OK;
}

static octmg_status set_leaf_field(octmg_state s, const void *src, int dtype, int on_device, hipStream_t st,
                                   int field) {
    octmg_geom g = s->geom;
    HIPCK(hipSetDevice(g->device));
    DevPool tmp(s->geom->allocator(), s->geom->device);
    double *dv = nullptr;
    const size_t n = (size_t)g->n_leaf * s->nrhs;
    STCK(stage_in_typed(src, dtype, n, on_device, st, &dv, &tmp));
    STCK(check_finite(s, dv, (long long)n, st));
    for (size_t il = 0; il < g->L.size(); il++) {
        const GeomLevel &L = g->L[il];
        HIPCK(launch_scatter_leaf(g->tree.D, L.Nb, lv64(s, (int)il), L.d_leaf_blocks, L.nleaf, dv, g->n_leaf,
                                  L.leaf_base, field, s->nrhs, st));
    }
    HIPCK(hipStreamSynchronize(st));
    return OCTMG_OK;
}

octmg_status octmg_set_rhs(octmg_state s, const void *gv, int dtype, int on_device, void *stream) {
    if (!s || !gv) return fail(OCTMG_ERR_INVALID, "null argument");
    STCK(check_dtype(dtype));
    s->r0_dirty = true;
    return set_leaf_field(s, gv, dtype, on_device, (hipStream_t)stream, 1);
}

octmg_status octmg_set_solution(octmg_state s, const void *phi, int dtype, int on_device, void *stream) {
    if (!s || !phi) return fail(OCTMG_ERR_INVALID, "null argument");
    STCK(check_dtype(dtype));
    return set_leaf_field(s, phi, dtype, on_device, (hipStream_t)stream, 0);
}

octmg_status octmg_get_solution(octmg_state s, void *phi, int dtype, int on_device, void *stream) {
    if (!s || !phi) return fail(OCTMG_ERR_INVALID, "null argument");
    STCK(check_dtype(dtype));
    hipStream_t st = (hipStream_t)stream;
    octmg_geom g = s->geom;
    HIPCK(hipSetDevice(g->device));
    const size_t n = (size_t)g->n_leaf * s->nrhs;
    DevPool tmp(s->geom->allocator(), s->geom->device);
    const bool f64 = dtype == OCTMG_DTYPE_F64;
    double *dv = (double *)phi;
    if (!on_device || !f64) HIPCK(tmp.alloc(&dv, n));
    for (size_t il = 0; il < g->L.size(); il++) {
        const GeomLevel &L = g->L[il];
        HIPCK(launch_gather_leaf(g->tree.D, L.Nb, lv64(s, (int)il), L.d_leaf_blocks, L.nleaf, dv, g->n_leaf,
                                 L.leaf_base, s->nrhs, st));
    }
    if (f64) {
        if (!on_device) HIPCK(hipMemcpyAsync(phi, dv, n * sizeof(double), hipMemcpyDeviceToHost, st));
    } else {
        // rounded to FP32 on the device, then copied if the caller's buffer is on the host
        float *df = (float *)phi;
        if (!on_device) HIPCK(tmp.alloc(&df, n));
        HIPCK(launch_copy_d2f(dv, df, (long long)n, st));
        if (!on_device) HIPCK(hipMemcpyAsync(phi, df, n * sizeof(float), hipMemcpyDeviceToHost, st));
    }
    HIPCK(hipStreamSynchronize(st));
    return OCTMG_OK;
}

octmg_status octmg_gradient(octmg_state s, int inside_zero, double *out, int on_device, void *stream) {
    if (!s || !out) return fail(OCTMG_ERR_INVALID, "null argument");
    hipStream_t st = (hipStream_t)stream;
    octmg_geom g = s->geom;
    HIPCK(hipSetDevice(g->device));
    Engine<double> e{s, st};
    STCK(e.sync_down());  // coarse copies of leaf values for refinement-boundary ghosts
    const size_t n = (size_t)3 * g->n_leaf * s->nrhs;
    DevPool tmp(s->geom->allocator(), s->geom->device);
    double *dv = out;
    if (!on_device) HIPCK(tmp.alloc(&dv, n));
    for (size_t il = 0; il < g->L.size(); il++) {
        const GeomLevel &L = g->L[il];
        LV<double> v = lv64(s, (int)il), vc = lv64(s, (int)il - 1);
        v.lanes = vc.lanes = nullptr;  // every rhs, grid y = rhs
        HIPCK(launch_gradient(g->tree.D, L.Nb, v, vc, L.d_leaf_blocks, L.nleaf, L.d_meta, L.d_d6, L.d_inside,
                              s->f64[il].pb, inside_zero, dv, 3LL * g->n_leaf, L.leaf_base, s->nrhs, st));
    }
    if (!on_device) HIPCK(hipMemcpyAsync(out, dv, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    return OCTMG_OK;
}

octmg_status octmg_state_remap(octmg_state from, octmg_state to, void *stream) {
    if (!from || !to) return fail(OCTMG_ERR_INVALID, "null argument");
    const octmg_geom go = from->geom, gn = to->geom;
    if (go->tree.D != gn->tree.D || go->tree.N != gn->tree.N || go->tree.nsub != gn->tree.nsub ||
        go->L.size() != gn->L.size() || from->nrhs != to->nrhs || go->device != gn->device)
        return fail(OCTMG_ERR_INVALID, "states of incompatible geometries");
    hipStream_t st = (hipStream_t)stream;
    HIPCK(hipSetDevice(gn->device));
    const int D = gn->tree.D, nlev = (int)gn->L.size();
    // every old cell, parent cells included, holds the mean of its leaves
    for (int il = nlev - 1; il > 0; il--) {
        LV<double> a = lv64(from, il), b = lv64(from, il - 1);
        a.lanes = b.lanes = nullptr;
        a.active = b.active = nullptr;
        HIPCK(launch_restrict_phi<double>(D, go->L[il].Nb, go->L[il - 1].Nb, a, b, from->nrhs, st));
    }
    std::vector<LV<double>> old(nlev);
    std::vector<int> nbo(nlev);
    for (int il = 0; il < nlev; il++) {
        old[il] = lv64(from, il);
        old[il].lanes = nullptr;
        old[il].active = nullptr;
        nbo[il] = go->L[il].Nb;
    }
    DevPool tmp(to->geom->allocator(), to->geom->device);
    LV<double> *d_old = nullptr;
    int *d_nb = nullptr;
    HIPCK(tmp.alloc(&d_old, (size_t)nlev));
    HIPCK(tmp.alloc(&d_nb, (size_t)nlev));
    HIPCK(hipMemcpyAsync(d_old, old.data(), sizeof(LV<double>) * nlev, hipMemcpyHostToDevice, st));
    HIPCK(hipMemcpyAsync(d_nb, nbo.data(), sizeof(int) * nlev, hipMemcpyHostToDevice, st));
    for (int il = 0; il < nlev; il++) {
        const GeomLevel &L = gn->L[il];
        HIPCK(launch_remap(D, L.Nb, lv64(to, il), il, d_old, d_nb, L.d_leaf_blocks, L.nleaf, to->nrhs, st));
    }
    Engine<double> e{to, st};
    STCK(e.sync_down());
    HIPCK(hipStreamSynchronize(st));
    return OCTMG_OK;
}

octmg_status octmg_zero_solution(octmg_state s, void *stream) {
    if (!s) return fail(OCTMG_ERR_INVALID, "null state");
    hipStream_t st = (hipStream_t)stream;
    HIPCK(hipSetDevice(s->geom->device));
    // on uniform trees only the leaf level is ever read before a cycle
    // overwrites it (restriction sets phi and old of coarser levels)
    const bool all = s->geom->tree.adaptive;
    for (size_t il = 0; il < s->f64.size(); il++) {
        if (!all && s->geom->L[il].nleaf == 0) continue;
        const long long n = s->stride[il] * s->nrhs;
        HIPCK(launch_fill(s->f64[il].phi, n, 0.0, st));
        if (all) HIPCK(launch_fill(s->f64[il].old, n, 0.0, st));
    }
    return OCTMG_OK;
}

octmg_status octmg_cycle(octmg_state s, int kind, int have_guess, void *stream) {
    if (!s) return fail(OCTMG_ERR_INVALID, "null state");
    if (kind != OCTMG_CYCLE_V && kind != OCTMG_CYCLE_FMG) return fail(OCTMG_ERR_INVALID, "bad cycle kind");
    hipStream_t st = (hipStream_t)stream;
    HIPCK(hipSetDevice(s->geom->device));
    if (s->precision == OCTMG_MIXED) {
        STCK(mixed_defect(s, st, kind == OCTMG_CYCLE_V));
        return mixed_correct(s, kind, st);
    }
    Engine<double> e{s, st};
    return e.cycle(kind, have_guess);
}

octmg_status octmg_residual_norm(octmg_state s, int phi_zero, double *out, void *stream) {
    if (!s || !out) return fail(OCTMG_ERR_INVALID, "null argument");
    hipStream_t st = (hipStream_t)stream;
    HIPCK(hipSetDevice(s->geom->device));
    STCK(residual_norm_dev(s, phi_zero, st));
    return read_norms(s, out, st);
}

// Flags and launch list in one upload: later launches cover only the
// iterating right-hand sides (grid y = their number), so finished or idle
// ones cost no workgroups.  With none iterating the list keeps every rhs
// (their kernels then exit at the flag) so that no launch is empty.
// With the pinned control buffers of a lane state (lanes_prepare) the upload
// is left in flight: the buffer it reads is not written again before the
// server's next pass, which waits for the stream first.
static octmg_status set_active(octmg_state s, const std::vector<int> &act, hipStream_t st) {
    std::vector<int> list;
    for (int r = 0; r < (int)act.size(); r++)
        if (act[r]) list.push_back(r);
    if (list.empty())
        for (int r = 0; r < (int)act.size(); r++) list.push_back(r);
    if (act == s->active_host && list == s->lanes_host) return OCTMG_OK;
    s->active_host = act;
    s->lanes_host = list;
    s->n_launch = (int)list.size();
    std::vector<int> ctrl(act);
    ctrl.insert(ctrl.end(), list.begin(), list.end());
    if (s->h_ctrl) {
        int *buf = s->h_ctrl + (size_t)s->ctrl_turn * 2 * s->nrhs;
        s->ctrl_turn ^= 1;
        std::memcpy(buf, ctrl.data(), sizeof(int) * ctrl.size());
        HIPCK(hipMemcpyAsync(s->d_active, buf, sizeof(int) * ctrl.size(), hipMemcpyHostToDevice, st));
        return OCTMG_OK;
    }
    HIPCK(hipMemcpyAsync(s->d_active, ctrl.data(), sizeof(int) * ctrl.size(), hipMemcpyHostToDevice, st));
    HIPCK(hipStreamSynchronize(st));
    return OCTMG_OK;
}

// One step of a solve after the convergence check: a cycle (or, in MIXED
// precision, the FP32 correction and the next FP64 defect), then the
// residual norms of the new iterate into d_norm and the mapped host buffer.
static octmg_status cycle_and_norm(octmg_state s, int kind, int have_guess, hipStream_t st) {
    if (s->precision == OCTMG_MIXED) {
        STCK(mixed_correct(s, kind, st));
        STCK(mixed_defect(s, st, kind == OCTMG_CYCLE_V));
    } else {
        Engine<double> e{s, st};
        STCK(e.cycle(kind, have_guess));
        STCK(residual_norm_dev(s, 0, st, true));
    }
    return OCTMG_OK;
}

extern "C++" {
// Capture `body` on stream st into an executable graph (cached under key).
template <typename F>
static octmg_status graph_for(octmg_state s, long long key, hipStream_t st, F &&body, hipGraphExec_t *out) {
    for (auto &kv : s->graphs)
        if (kv.first == key) {
            *out = kv.second;
            return OCTMG_OK;
        }
    // profiling events and counters cover eager launches only
    const bool prof_on = s->prof && s->prof->on;
    if (prof_on) s->prof->on = false;
    // capturing runs no kernel: the state of the norm slots is unchanged
    const bool slots_clean = s->norm_slots_clean;
    HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const octmg_status r = body();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (prof_on) s->prof->on = true;
    s->norm_slots_clean = slots_clean;
    if (r != OCTMG_OK) {
        if (e == hipSuccess && g) (void)hipGraphDestroy(g);
        return r;
    }
    HIPCK(e);
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCK(ei);
    s->graphs.push_back({key, exec});
    *out = exec;
    return OCTMG_OK;
}

}  // extern "C++"

// cache key of a captured graph: what it was captured for, including the
// number of grid rows of its launches
static long long graph_key(int mode, int kind, int max_cycles, int zero_start, int n_launch) {
    // (graph_mode 2 appends its chunk length: key * 128 + K)
    return ((((long long)mode * 8 + kind) * 128 + max_cycles) * 4 + zero_start) * 8192 + n_launch;
}

// after the stream has passed the norm kernel
static octmg_status read_mapped(octmg_state s, std::vector<double> &out, hipStream_t st) {
    if (!s->h_norm) return read_norms(s, out.data(), st);
    for (int r = 0; r < s->nrhs; r++) {
        const unsigned long long v = ((volatile unsigned long long *)s->h_norm)[r];
        std::memcpy(&out[r], &v, sizeof(double));
    }
    return OCTMG_OK;
}

// Cycles until every right-hand side satisfies max|r| <= rtol * max|r(0)|.
// A right-hand side that has converged is frozen (its kernels exit early),
// so each one receives exactly the cycles a solve of it alone would.
// graph_mode 0: eager launches; 1: each cycle replays one captured graph;
// 2: the whole solve is one captured graph of max_cycles cycles, with the
// convergence test on the device (no stall test in that mode).
// Outcome of each right-hand side of a solve: cycles it received, its last
// residual norm, and whether it reached rtol.
struct PerRhs {
    std::vector<int> cycles, done;
    std::vector<double> r0, r_final;
};

static octmg_status solve_impl(octmg_state s, const octmg_solve_opts *o, hipStream_t st, octmg_solve_report *rp,
                               PerRhs &pr) {
    const int R = s->nrhs;
    std::vector<double> r0(R), rk(R), prev(R, 0.0);
    std::vector<double> &cur = pr.r_final;
    std::vector<int> act(R, 1);
    cur.assign(R, 0.0);
    pr.cycles.assign(R, 0);
    pr.done.assign(R, 0);
    STCK(set_active(s, act, st));
    if (s->r0_dirty) {
        STCK(residual_norm_dev(s, 1, st));
        STCK(read_norms(s, r0.data(), st));
        s->r0_cache = r0;
        s->r0_dirty = false;
    }
    r0 = s->r0_cache;
    pr.r0 = r0;
    if (o->zero_start) STCK(octmg_zero_solution(s, st));
    std::memset(rp, 0, offsetof(octmg_solve_report, rhs_status));
    for (double v : r0) rp->r0 = std::max(rp->r0, v);
    // residual of the starting iterate
    if (s->precision == OCTMG_MIXED) {
        STCK(mixed_defect(s, st, o->cycle_kind == OCTMG_CYCLE_V));
        STCK(read_norms(s, rk.data(), st));
    } else if (o->zero_start) {
        rk = r0;  // the residual of phi = 0 is r0 itself
    } else {
        STCK(residual_norm_dev(s, 0, st));
        STCK(read_norms(s, rk.data(), st));
    }
    if (o->graph_mode == 2) {
        // everything after the first check runs inside one graph
        bool all_done = true;
        std::vector<double> th(R);
        for (int r = 0; r < R; r++) {
            cur[r] = rk[r];
            th[r] = o->rtol * r0[r];
            if (!(rk[r] <= th[r])) all_done = false;
            act[r] = rk[r] <= th[r] ? 0 : 1;
            pr.done[r] = 1 - act[r];
            rp->r_final = std::max(rp->r_final, rk[r]);
        }
        if (all_done) {
            rp->status = OCTMG_OK;
            return OCTMG_OK;
        }
        STCK(set_active(s, act, st));
        HIPCK(hipMemcpyAsync(s->d_thresh, th.data(), sizeof(double) * R, hipMemcpyHostToDevice, st));
        // The cycles run as replays of captured chunks of cycles, each cycle
        // followed by its convergence test; the host looks at the running
        // flags after each chunk and stops once none runs.  The first chunk
        // has as many cycles as the state's last solve took (else all
        // max_cycles of them when that is at most 16, else 8), the later
        // ones one cycle each.  The cycles of a chunk after every rhs has
        // stopped launch and exit at once.
        const int K1 = std::min(o->max_cycles, s->cycle_hint > 0 ? s->cycle_hint
                                                                 : (o->max_cycles <= 16 ? o->max_cycles : 8));
        HIPCK(hipMemsetAsync(s->d_cbase, 0, sizeof(int), st));  // outside the graphs
        std::vector<int> act_after(R);
        for (int launched = 0, K = K1; launched < o->max_cycles; launched += K, K = 1) {
            const bool first = launched == 0;
            // the first chunk starts from the caller's iterate (an FMG's
            // first cycle without a guess when zero_start); later ones go on
            const long long key =
                graph_key(2, o->cycle_kind, o->max_cycles, first ? (o->zero_start ? 1 : 0) : 2, s->n_launch) * 128 + K;
            hipGraphExec_t exec = nullptr;
            STCK(graph_for(s, key, st, [&]() -> octmg_status {
                for (int c = 0; c < K; c++) {
                    STCK(cycle_and_norm(s, o->cycle_kind, (c > 0 || !first || !o->zero_start) ? 1 : 0, st));
                    HIPCK(launch_converge(s->d_norm, s->d_thresh, s->d_active, s->d_hist, c, R, s->d_cbase,
                                          o->max_cycles, c == K - 1 ? K : 0, st));
                }
                return OCTMG_OK;
            }, &exec));
            STCK(clean_norm_slots(s, st));
            HIPCK(hipGraphLaunch(exec, st));
            HIPCK(hipMemcpyAsync(act_after.data(), s->d_active, sizeof(int) * R, hipMemcpyDeviceToHost, st));
            HIPCK(hipStreamSynchronize(st));
            bool running = false;
            for (int r = 0; r < R; r++) running |= act_after[r] != 0;
            if (!running) break;
        }
        std::vector<double> hist((size_t)o->max_cycles * R);
        HIPCK(hipMemcpyAsync(hist.data(), s->d_hist, sizeof(double) * hist.size(), hipMemcpyDeviceToHost, st));
        HIPCK(hipStreamSynchronize(st));
        s->active_host = act_after;
        int cycles = 0;
        bool nonfinite = false;
        for (int c = 0; c < o->max_cycles; c++) {
            double rmax = 0.0;
            bool any = false;
            for (int r = 0; r < R; r++) {
                if (!act[r]) continue;  // converged before this cycle
                cur[r] = hist[(size_t)c * R + r];
                pr.cycles[r] = c + 1;
                if (!std::isfinite(cur[r])) nonfinite = true;
                if (cur[r] <= th[r]) act[r] = 0, pr.done[r] = 1;
                any = true;
            }
            if (!any) break;
            for (int r = 0; r < R; r++) rmax = std::max(rmax, cur[r]);
            rp->history[c] = rmax;
            cycles = c + 1;
            rp->r_final = rmax;
        }
        rp->cycles = cycles;
        bool done = true;
        for (int r = 0; r < R; r++)
            if (act[r]) done = false;
        if (nonfinite) {
            rp->status = OCTMG_ERR_NONFINITE;
            return fail(OCTMG_ERR_NONFINITE, "residual became non-finite");
        }
        rp->status = done ? OCTMG_OK : OCTMG_ERR_NOT_CONVERGED;
        return done ? OCTMG_OK : fail(OCTMG_ERR_NOT_CONVERGED, "rtol not reached");
    }
    int stall = 0;
    bool have_guess = !o->zero_start;
    for (int k = 0; k <= o->max_cycles; k++) {
        bool all_done = true, nonfinite = false, changed = false;
        double rmax = 0.0;
        for (int r = 0; r < R; r++) {
            if (act[r]) cur[r] = rk[r];
            if (!std::isfinite(cur[r])) nonfinite = true;
            rmax = std::max(rmax, cur[r]);
            if (act[r]) pr.cycles[r] = k;
            if (act[r] && cur[r] <= o->rtol * r0[r]) {
                act[r] = 0;
                pr.done[r] = 1;
                changed = true;
            }
            if (act[r]) all_done = false;
        }
        if (k > 0 && k <= 64) rp->history[k - 1] = rmax;
        rp->cycles = k;
        rp->r_final = rmax;
        if (nonfinite) {
            rp->status = OCTMG_ERR_NONFINITE;
            return fail(OCTMG_ERR_NONFINITE, "residual became non-finite");
        }
        if (all_done) {
            rp->status = OCTMG_OK;
            return OCTMG_OK;
        }
        if (k == o->max_cycles) break;
        if (k > 0) {
            bool slow = true;
            for (int r = 0; r < R; r++)
                if (act[r] && !(cur[r] > 0.95 * prev[r])) slow = false;
            stall = slow ? stall + 1 : 0;
            if (stall >= 3) break;
        }
        prev = cur;
        if (changed) STCK(set_active(s, act, st));
        if (o->graph_mode == 1 && have_guess) {
            const long long key = graph_key(1, o->cycle_kind, 0, 0, s->n_launch);
            hipGraphExec_t exec = nullptr;
            STCK(graph_for(s, key, st, [&]() { return cycle_and_norm(s, o->cycle_kind, 1, st); }, &exec));
            STCK(clean_norm_slots(s, st));
            HIPCK(hipGraphLaunch(exec, st));
        } else {
            STCK(cycle_and_norm(s, o->cycle_kind, have_guess ? 1 : 0, st));
        }
        HIPCK(hipStreamSynchronize(st));
        STCK(read_mapped(s, rk, st));
        have_guess = true;
    }
    rp->status = OCTMG_ERR_NOT_CONVERGED;
    return fail(OCTMG_ERR_NOT_CONVERGED, "rtol not reached");
}

octmg_status octmg_solve(octmg_state s, const octmg_solve_opts *o, void *stream, octmg_solve_report *rep) {
    if (!s || !o) return fail(OCTMG_ERR_INVALID, "null argument");
    if (!(o->rtol > 0.0) || o->max_cycles < 1 || o->max_cycles > 64) return fail(OCTMG_ERR_INVALID, "bad options");
    if (o->cycle_kind != OCTMG_CYCLE_V && o->cycle_kind != OCTMG_CYCLE_FMG) return fail(OCTMG_ERR_INVALID, "bad cycle kind");
    if (o->graph_mode < 0 || o->graph_mode > 2) return fail(OCTMG_ERR_INVALID, "bad graph_mode");
    hipStream_t st = (hipStream_t)stream;
    HIPCK(hipSetDevice(s->geom->device));
    if (o->graph_mode && s->fused_top >= 1) return fail(OCTMG_ERR_INVALID, "graph capture needs fused levels off");
    if (o->graph_mode && !st) {
        // the legacy default stream cannot be captured: use a blocking stream
        // of the state, which orders itself with the default stream
        if (!s->own_stream) HIPCK(hipStreamCreate(&s->own_stream));
        st = s->own_stream;
    }
    octmg_solve_report local{};
    PerRhs pr;
    octmg_status res = solve_impl(s, o, st, rep ? rep : &local, pr);
    std::string msg = g_last_error;
    // the next solve's first graph chunk (graph_mode 2) covers as many cycles
    // as this one took, if it converged (else the default chunk: a solve cut
    // off at max_cycles would make the next one launch that many)
    s->cycle_hint = res == OCTMG_OK ? (rep ? rep : &local)->cycles : 0;
    if (rep && (int)pr.r_final.size() == s->nrhs)
        for (int r = 0; r < s->nrhs; r++) {
            const bool finite = std::isfinite(pr.r_final[r]);
            if (rep->rhs_status)
                rep->rhs_status[r] = !finite ? OCTMG_ERR_NONFINITE : pr.done[r] ? OCTMG_OK : OCTMG_ERR_NOT_CONVERGED;
            if (rep->rhs_cycles) rep->rhs_cycles[r] = pr.cycles[r];
            if (rep->rhs_r0) rep->rhs_r0[r] = pr.r0.empty() ? 0.0 : pr.r0[r];
            if (rep->rhs_r_final) rep->rhs_r_final[r] = pr.r_final[r];
        }
    std::vector<int> all(s->nrhs, 1);
    STCK(set_active(s, all, st));
    if (res != OCTMG_OK) return fail(res, msg);
    return OCTMG_OK;
}

// Tune-cache key of a state's problem: everything the launch choice depends
// on (device, tree shape, records, right-hand sides, precision, options).
static std::string tune_key(octmg_state s, const octmg_solve_opts *o) {
    hipDeviceProp_t prop{};
    (void)hipGetDeviceProperties(&prop, s->geom->device);
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s cu%d D%d N%d rec%lld rhs%d prec%d kind%d rtol%.3e max%d", prop.gcnArchName,
                  prop.multiProcessorCount, s->geom->tree.D, s->geom->tree.N, s->geom->n_rec, s->nrhs, s->precision,
                  o->cycle_kind, o->rtol, o->max_cycles);
    std::string k(buf);
    for (const GeomLevel &L : s->geom->L) k += " " + std::to_string(L.nblocks) + "/" + std::to_string(L.nleaf);
    return k;
}

static std::mutex g_tune_mu;  // one writer of a tune-cache file at a time in this process

// the launch configuration recorded for `key` (the last such line wins)
static bool tune_lookup(const std::string &path, const std::string &key, octmg_launch_config *c) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    bool found = false;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        char *tab = std::strchr(line, '\t');
        if (!tab || std::string(line, tab - line) != key) continue;
        octmg_launch_config t{};
        if (std::sscanf(tab + 1, "%d %d %d %d %d %d %d %d", &t.block_order, &t.bottom_kind, &t.bottom_max_blocks,
                        &t.graph_mode, &t.pair_max_blocks, &t.prolong_fused, &t.red_preset, &t.update_fused) == 8) {
            *c = t;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

static void tune_record(const std::string &path, const std::string &key, const octmg_launch_config &c, double ms) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;  // an unwritable cache only costs the next tuning run
    std::fprintf(f, "%s\t%d %d %d %d %d %d %d %d %.4f\n", key.c_str(), c.block_order, c.bottom_kind,
                 c.bottom_max_blocks, c.graph_mode, c.pair_max_blocks, c.prolong_fused, c.red_preset, c.update_fused,
                 ms);
    std::fclose(f);
}

octmg_status octmg_autotune(octmg_state s, const octmg_solve_opts *o, int reps, void *stream,
                            octmg_launch_config *best, double *ms, int *n_candidates) {
    if (!s || !o || !best || reps < 1) return fail(OCTMG_ERR_INVALID, "bad argument");
    const octmg_ctx ctx = s->geom->ctx;
    const bool cached = ctx && !ctx->tune_path.empty();
    const std::string key = cached ? tune_key(s, o) : std::string();
    if (cached && tune_lookup(ctx->tune_path, key, best)) {
        if (n_candidates) *n_candidates = 0;
        return octmg_state_set_launch(s, best);
    }
    std::vector<octmg_launch_config> cand;
    constexpr int all = 1 << 30;
    for (int order = 0; order < 3; order++) {
        cand.push_back({order, 0, 0, 0, all, 1, 1, 1});
        cand.push_back({order, 0, 0, 1, all, 1, 1, 1});
        if (s->geom->tree.D == 3) {
            cand.push_back({order, 1, 8, 0, all, 1, 1, 1});
            cand.push_back({order, 1, 64, 0, all, 1, 1, 1});
        }
    }
    if (s->geom->tree.D == 3) {
        cand.push_back({0, 0, 0, 0, 0, 1, 1, 1});
        cand.push_back({0, 0, 0, 1, 0, 1, 1, 1});
    }
    // the whole solve as one captured launch (max_cycles cycles, convergence
    // tested on the device), with the 512- and the 256-thread kernels
    cand.push_back({0, 0, 0, 2, all, 1, 1, 1});
    if (s->geom->tree.D == 3) cand.push_back({0, 0, 0, 2, 0, 1, 1, 1});
    if (n_candidates) *n_candidates = (int)cand.size();
    double best_ms = 0.0;
    int best_i = -1;
    for (size_t i = 0; i < cand.size(); i++) {
        STCK(octmg_state_set_launch(s, &cand[i]));
        octmg_solve_opts so = *o;
        so.zero_start = 1;
        so.graph_mode = cand[i].graph_mode;
        octmg_solve_report rep{};
        STCK(octmg_solve(s, &so, stream, &rep));  // warm: captures graphs, fills caches
        const auto t0 = std::chrono::steady_clock::now();
        for (int r = 0; r < reps; r++) STCK(octmg_solve(s, &so, stream, &rep));
        const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / reps;
        if (ms) ms[i] = t;
        if (best_i < 0 || t < best_ms) best_ms = t, best_i = (int)i;
    }
    *best = cand[best_i];
    if (cached) tune_record(ctx->tune_path, key, *best, best_ms);
    return octmg_state_set_launch(s, best);
}

octmg_status octmg_debug_get_field(octmg_state s, int level, int field, int rhs, double *out) {
    STCK(check_level(s, level));
    if (rhs < 0 || rhs >= s->nrhs || !out || field < 0 || field > 2) return fail(OCTMG_ERR_INVALID, "bad argument");
    HIPCK(hipSetDevice(s->geom->device));
    const GeomLevel &L = s->geom->L[level];
    const Fields64 &F = s->f64[level];
    double *src = (field == 0 ? F.phi : field == 1 ? F.g : F.old) + s->stride[level] * rhs;
    const size_t n = (size_t)L.nblocks * L.cpb;
    DevPool tmp(s->geom->allocator(), s->geom->device);
    double *canon = nullptr;
    HIPCK(tmp.alloc(&canon, n));
    HIPCK(launch_level_copy(s->geom->tree.D, L.Nb, src, canon, L.nblocks, 0, nullptr));
    HIPCK(hipMemcpy(out, canon, n * sizeof(double), hipMemcpyDeviceToHost));
    return OCTMG_OK;
}

octmg_status octmg_debug_set_field(octmg_state s, int level, int field, int rhs, const double *in) {
    STCK(check_level(s, level));
    if (rhs < 0 || rhs >= s->nrhs || !in || field < 0 || field > 2) return fail(OCTMG_ERR_INVALID, "bad argument");
    HIPCK(hipSetDevice(s->geom->device));
    const GeomLevel &L = s->geom->L[level];
    const Fields64 &F = s->f64[level];
    double *dst = (field == 0 ? F.phi : field == 1 ? F.g : F.old) + s->stride[level] * rhs;
    const size_t n = (size_t)L.nblocks * L.cpb;
    DevPool tmp(s->geom->allocator(), s->geom->device);
    double *canon = nullptr;
    HIPCK(tmp.alloc(&canon, n));
    HIPCK(hipMemcpy(canon, in, n * sizeof(double), hipMemcpyHostToDevice));
    HIPCK(launch_level_copy(s->geom->tree.D, L.Nb, dst, canon, L.nblocks, 1, nullptr));
    HIPCK(hipDeviceSynchronize());
    return OCTMG_OK;
}

octmg_status octmg_debug_step(octmg_state s, int step, int level, int arg, void *stream) {
    if (!s) return fail(OCTMG_ERR_INVALID, "null state");
    hipStream_t st = (hipStream_t)stream;
    HIPCK(hipSetDevice(s->geom->device));
    Engine<double> e{s, st};
    const int nlev = (int)s->geom->L.size();
    if (step != OCTMG_STEP_COARSE_SOLVE) STCK(check_level(s, level));
    switch (step) {
        case OCTMG_STEP_HALF_SWEEP:
            if (arg != 0 && arg != 1) return fail(OCTMG_ERR_INVALID, "colour must be 0 or 1");
            STCK(e.half_sweep(level, arg));
            break;
        case OCTMG_STEP_SMOOTH:
            STCK(e.smooth(level, arg));
            break;
        case OCTMG_STEP_RESTRICT_FAS:
            if (level < 1) return fail(OCTMG_ERR_INVALID, "level must be >= 1");
            STCK(e.restrict_fas(level));
            break;
        case OCTMG_STEP_PROLONG:
            if (level < 1) return fail(OCTMG_ERR_INVALID, "level must be >= 1");
            STCK(e.prolong(level, arg));
            break;
        case OCTMG_STEP_COARSE_SOLVE:
            STCK(e.coarse_solve());
            break;
        case OCTMG_STEP_RESTRICT_RHS:
            if (level < 1) return fail(OCTMG_ERR_INVALID, "level must be >= 1");
            STCK(e.restrict_rhs(level));
            break;
        default:
            return fail(OCTMG_ERR_INVALID, "unknown step");
    }
    (void)nlev;
    HIPCK(hipStreamSynchronize(st));
    return OCTMG_OK;
}

// ------------------------------------------------- allocation-free solve
// octmg_solve_noalloc keeps every field of its one-rhs FP64 solve in this
// array of the library's device code, one copy per device, which lives as
// long as the process.  Its address on a device is looked up once, with that
// device current, and only that address is used from host code.
constexpr size_t kNoallocBytes = size_t(64) << 20;
constexpr int kNoallocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kNoallocMaxDevices] = {};

// the current device's copy of `scratch`
static octmg_status scratch_on(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kNoallocMaxDevices) return fail(OCTMG_ERR_INVALID, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(OCTMG_ERR_HIP, "no device address for the scratch array");
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[dev];
    return OCTMG_OK;
}

extern "C++" {
// bump allocation of 256-byte aligned pieces of the scratch array
struct ScratchCut {
    uintptr_t base;
    size_t used = 0;
    template <typename T>
    T *take(size_t n) {
        T *p = (T *)(base + used);
        used += (n * sizeof(T) + 255) / 256 * 256;
        return p;
    }
};

// bytes of the scratch array that a solve on g needs
static size_t noalloc_bytes(octmg_geom g) {
    ScratchCut c{0};
    const int D = g->tree.D;
    for (const GeomLevel &L : g->L) {
        const size_t cells = (size_t)L.nblocks * L.cpb;
        for (int f = 0; f < 3; f++) c.take<double>(cells);
        c.take<double>(std::max(1, L.nrec));
        c.take<double>((size_t)2 * D * L.nface);
    }
    c.take<unsigned long long>(1);
    c.take<unsigned long long>((size_t)norm_slot_words(1));
    c.take<int>(1);
    c.take<int>(2);
    return c.used;
}
}  // extern "C++"

octmg_status octmg_solve_noalloc(octmg_geom g, const double *rhs, const double *iface_vals, const double *domain_vals,
                                 double *phi, const octmg_solve_opts *o, void *stream, octmg_solve_report *rep) {
    if (!g || !rhs || !phi || !o) return fail(OCTMG_ERR_INVALID, "null argument");
    if (!(o->rtol > 0.0) || o->max_cycles < 1 || o->max_cycles > 64) return fail(OCTMG_ERR_INVALID, "bad options");
    if (o->cycle_kind != OCTMG_CYCLE_V && o->cycle_kind != OCTMG_CYCLE_FMG) return fail(OCTMG_ERR_INVALID, "bad cycle kind");
    if (o->graph_mode != 0) return fail(OCTMG_ERR_INVALID, "octmg_solve_noalloc launches eagerly: graph_mode must be 0");
    const size_t need = noalloc_bytes(g);
    if (need > kNoallocBytes)
        return fail(OCTMG_ERR_INVALID, "geometry too large for octmg_solve_noalloc: its fields need " +
                                           std::to_string(need) + " bytes, the scratch array holds " +
                                           std::to_string(kNoallocBytes));
    hipStream_t st = (hipStream_t)stream;
    HIPCK(hipSetDevice(g->device));
    unsigned char *base = nullptr;
    STCK(scratch_on(g->device, &base));

    // a one-rhs FP64 state whose device memory is all in the scratch array
    octmg_state_s s;
    s.geom = g;
    const int nlev = (int)g->L.size(), D = g->tree.D;
    s.f64.resize(nlev);
    s.stride.resize(nlev);
    ScratchCut c{(uintptr_t)base};
    for (int il = 0; il < nlev; il++) {
        const GeomLevel &L = g->L[il];
        const long long cells = (long long)L.nblocks * L.cpb;
        s.stride[il] = cells;
        Fields64 &F = s.f64[il];
        F.phi = c.take<double>(cells);
        F.g = c.take<double>(cells);
        F.old = c.take<double>(cells);
        F.b = c.take<double>(std::max(1, L.nrec));
        F.bcv = c.take<double>((size_t)2 * D * L.nface);
    }
    s.d_norm = c.take<unsigned long long>(1);
    s.d_norm_slots = c.take<unsigned long long>((size_t)norm_slot_words(1));
    s.d_flag = c.take<int>(1);
    s.d_active = c.take<int>(2);
    s.h_norm_dev = s.d_norm;  // no mapped host buffer: norms are copied back
    s.norm_slots_clean = false;

    // every field starts at zero, as in a new state (the array keeps the
    // previous call's values)
    for (int il = 0; il < nlev; il++) {
        const GeomLevel &L = g->L[il];
        Fields64 &F = s.f64[il];
        HIPCK(launch_fill(F.phi, s.stride[il], 0.0, st));
        HIPCK(launch_fill(F.g, s.stride[il], 0.0, st));
        HIPCK(launch_fill(F.old, s.stride[il], 0.0, st));
        HIPCK(launch_fill(F.b, std::max(1, L.nrec), 0.0, st));
    }
    // boundary data (as octmg_set_boundary) and rhs (as octmg_set_rhs)
    if (iface_vals && g->n_pts) STCK(check_finite(&s, iface_vals, g->n_pts, st));
    if (domain_vals) STCK(check_finite(&s, domain_vals, g->n_dom, st));
    STCK(check_finite(&s, rhs, g->n_leaf, st));
    long long dom_off = 0;
    for (int il = 0; il < nlev; il++) {
        const GeomLevel &L = g->L[il];
        Fields64 &F = s.f64[il];
        HIPCK(launch_boundary_terms(D, L.d_meta, L.d_cfull, L.nrec, iface_vals ? iface_vals + L.pt_base : nullptr,
                                    F.b, nullptr, st));
        const long long nf = 2LL * D * L.nface;
        if (domain_vals)
            HIPCK(hipMemcpyAsync(F.bcv, domain_vals + dom_off, nf * sizeof(double), hipMemcpyDeviceToDevice, st));
        else
            HIPCK(launch_fill(F.bcv, nf, 0.0, st));
        dom_off += nf;
        HIPCK(launch_scatter_leaf(D, L.Nb, lv64(&s, il), L.d_leaf_blocks, L.nleaf, rhs, g->n_leaf, L.leaf_base, 1, 1,
                                  st));
    }
    octmg_solve_opts so = *o;
    so.zero_start = 1;
    octmg_solve_report local{};
    PerRhs pr;
    const octmg_status res = solve_impl(&s, &so, st, rep ? rep : &local, pr);
    const std::string msg = g_last_error;
    if (rep && pr.r_final.size() == 1) {
        if (rep->rhs_status)
            rep->rhs_status[0] = !std::isfinite(pr.r_final[0]) ? OCTMG_ERR_NONFINITE
                                 : pr.done[0]                  ? OCTMG_OK
                                                               : OCTMG_ERR_NOT_CONVERGED;
        if (rep->rhs_cycles) rep->rhs_cycles[0] = pr.cycles[0];
        if (rep->rhs_r0) rep->rhs_r0[0] = pr.r0.empty() ? 0.0 : pr.r0[0];
        if (rep->rhs_r_final) rep->rhs_r_final[0] = pr.r_final[0];
    }
    if (res == OCTMG_OK || res == OCTMG_ERR_NOT_CONVERGED)
        for (int il = 0; il < nlev; il++) {
            const GeomLevel &L = g->L[il];
            HIPCK(launch_gather_leaf(D, L.Nb, lv64(&s, il), L.d_leaf_blocks, L.nleaf, phi, g->n_leaf, L.leaf_base, 1,
                                     st));
        }
    HIPCK(hipStreamSynchronize(st));
    if (res != OCTMG_OK) return fail(res, msg);
    return OCTMG_OK;
}

}  // extern "C"

// ------------------------------------------------- lanes (serving engine)
// A lane is one right-hand side of a multi-rhs state.  These calls touch only
// the lanes they are given; the serving engine batches independent requests
// on one geometry by giving each its own lane.
namespace octmg {

octmg_status api_fail(octmg_status st, const std::string &msg) { return fail(st, msg); }

int geom_device(octmg_geom g) { return g->device; }

// what octmg_state_create allocates per right-hand side: phi, g, old on all
// levels (plus their FP32 copies in MIXED precision), the norm, its slots,
// the threshold, the graph history and two control words
size_t lane_bytes(octmg_geom g, int precision) {
    size_t cells = 0;
    for (const GeomLevel &L : g->L) cells += (size_t)L.nblocks * L.cpb;
    const size_t nf = g->tree.D == 3 ? 4 : 3;  // phi, g, old (and bp in 3D)
    return cells * (nf * sizeof(double) + (precision == OCTMG_MIXED ? nf * sizeof(float) : 0)) +
           (1 + (size_t)norm_slot_words(1) + 1 + 64) * sizeof(double) + 2 * sizeof(int);
}

// and once per state: boundary terms, face values and interface values of
// every level, the flag, plus one leaf-ordered staging buffer (a request
// with host buffers is staged through it)
size_t state_fixed_bytes(octmg_geom g) {
    size_t n = 1;
    for (const GeomLevel &L : g->L)
        n += (size_t)std::max(1, L.nrec) + (size_t)2 * g->tree.D * L.nface + (size_t)std::max<long long>(1, L.npts);
    return n * sizeof(double) + (size_t)g->n_leaf * sizeof(double);
}

static LV<double> lv64_lane(const octmg_state_s *s, int il, int lane) {
    LV<double> v = lv64(s, il);
    const long long o = (long long)lane * s->stride[il];
    v.phi += o;
    v.g += o;
    v.old += o;
    v.active += lane;
    v.lanes = nullptr;
    return v;
}

octmg_status lanes_prepare(octmg_state s) {
    if (s->h_ctrl) return OCTMG_OK;
    HIPCK(hipSetDevice(s->geom->device));
    HIPCK(hipHostMalloc((void **)&s->h_ctrl, sizeof(int) * 4 * s->nrhs, hipHostMallocDefault));
    HIPCK(hipHostMalloc((void **)&s->h_begin, sizeof(unsigned long long) * 2 * s->nrhs, hipHostMallocMapped));
    HIPCK(hipHostGetDevicePointer((void **)&s->h_begin_dev, s->h_begin, 0));
    return OCTMG_OK;
}

octmg_status lane_load(octmg_state s, int lane, const double *src, int on_device, hipStream_t st) {
    if (lane < 0 || lane >= s->nrhs) return fail(OCTMG_ERR_INVALID, "lane out of range");
    octmg_geom g = s->geom;
    DevPool tmp(s->geom->allocator(), s->geom->device);
    double *dv = nullptr;
    STCK(stage_in(src, (size_t)g->n_leaf, on_device, st, &dv, &tmp));
    for (size_t il = 0; il < g->L.size(); il++) {
        const GeomLevel &L = g->L[il];
        const long long o = (long long)lane * s->stride[il];
        HIPCK(launch_fill(s->f64[il].phi + o, s->stride[il], 0.0, st));
        HIPCK(launch_fill(s->f64[il].old + o, s->stride[il], 0.0, st));
        LV<double> v = lv64_lane(s, (int)il, lane);
        v.active = nullptr;
        HIPCK(launch_scatter_leaf(g->tree.D, L.Nb, v, L.d_leaf_blocks, L.nleaf, dv, g->n_leaf, L.leaf_base, 1, 1,
                                  st));
    }
    if (!on_device) HIPCK(hipStreamSynchronize(st));  // the staging buffer dies here
    return OCTMG_OK;
}

octmg_status lane_store(octmg_state s, int lane, double *dst, int on_device, hipStream_t st) {
    if (lane < 0 || lane >= s->nrhs) return fail(OCTMG_ERR_INVALID, "lane out of range");
    octmg_geom g = s->geom;
    DevPool tmp(s->geom->allocator(), s->geom->device);
    double *dv = dst;
    if (!on_device) HIPCK(tmp.alloc(&dv, (size_t)g->n_leaf));
    for (size_t il = 0; il < g->L.size(); il++) {
        const GeomLevel &L = g->L[il];
        LV<double> v = lv64_lane(s, (int)il, lane);
        v.active = nullptr;
        HIPCK(launch_gather_leaf(g->tree.D, L.Nb, v, L.d_leaf_blocks, L.nleaf, dv, g->n_leaf, L.leaf_base, 1, st));
    }
    if (!on_device) {
        HIPCK(hipMemcpyAsync(dst, dv, sizeof(double) * g->n_leaf, hipMemcpyDeviceToHost, st));
        HIPCK(hipStreamSynchronize(st));
    }
    return OCTMG_OK;
}

// Residual of phi = 0 and the first convergence norm (FP64: the same; MIXED:
// the first defect) of the lanes set in `fresh` into the state's begin
// buffers; lanes not in `fresh` keep their fields.  Read with
// lanes_begin_norms once the stream has passed.
octmg_status lanes_begin(octmg_state s, const std::vector<int> &fresh, hipStream_t st) {
    STCK(set_active(s, fresh, st));
    STCK(residual_norm_dev(s, 1, st, false, s->h_begin_dev));
    if (s->precision == OCTMG_MIXED) STCK(mixed_defect(s, st, true, s->h_begin_dev + s->nrhs));
    return OCTMG_OK;
}

void lanes_begin_norms(octmg_state s, std::vector<double> &r0, std::vector<double> &rk) {
    r0.resize(s->nrhs);
    rk.resize(s->nrhs);
    for (int r = 0; r < s->nrhs; r++) {
        const unsigned long long a = ((volatile unsigned long long *)s->h_begin)[r];
        const unsigned long long b = ((volatile unsigned long long *)s->h_begin)[s->nrhs + r];
        std::memcpy(&r0[r], &a, sizeof(double));
        std::memcpy(&rk[r], s->precision == OCTMG_MIXED ? &b : &a, sizeof(double));
    }
}

// Launch one cycle of the lanes set in `running` and the norms of the new
// iterates into the host-mapped buffer; returns without waiting.
octmg_status lanes_cycle(octmg_state s, const std::vector<int> &running, int kind, hipStream_t st) {
    STCK(set_active(s, running, st));
    const long long key = graph_key(1, kind, 0, 0, s->n_launch);
    hipGraphExec_t exec = nullptr;
    STCK(graph_for(s, key, st, [&]() { return cycle_and_norm(s, kind, 1, st); }, &exec));
    STCK(clean_norm_slots(s, st));
    HIPCK(hipGraphLaunch(exec, st));
    return OCTMG_OK;
}

void lanes_norms(octmg_state s, std::vector<double> &out) {
    out.resize(s->nrhs);
    (void)read_mapped(s, out, nullptr);  // lane states have the mapped buffer: no copy
}

}  // namespace octmg
