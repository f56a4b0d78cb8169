// HIP kernels of the multigrid cycle for gfx950 (CDNA4, wave64).
//
// One workgroup owns one block of N^D cells (N = 8 or 16).  Fields use the
// colour-split block-major layout described in octmg_internal.hpp, so a
// red-black half-sweep touches each HBM byte once: the other colour's phi
// (read), this colour's g (read) and this colour's phi (written).  Ghost
// values are never stored; they are formed where a neighbour is read:
//   same level      -> the neighbour block's cell (level lookup table)
//   domain face     -> 2 phi_b(face centre) - phi_inside (Dirichlet), or
//                      phi_inside (zero flux)
//   refinement edge -> 1/2 C_k + 3/4 f1 - 1/4 f2, C_k = C + sum_t s_t
//                      (C_t+ - C_t-)/8 from the next coarser level, which
//                      makes the coarse flux equal the averaged fine flux.
// Cells near the interface carry their own stencil (record index per cell,
// Sec. 3.6.2); every other cell uses the constant 2D+1 point Laplacian.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "octmg_internal.hpp"

namespace octmg {
namespace {

template <int D, int N>
struct Blk {
    static constexpr int NH = N / 2;
    static constexpr int CPB = D == 3 ? N * N * N : N * N;
    static constexpr int HALF = CPB / 2;
    static constexpr int THREADS = HALF >= 256 ? 256 : (HALF >= 64 ? HALF : 64);
};

template <int D, int N>
__device__ __forceinline__ int split_of(int i, int j, int k) {
    return ((i + j + k) & 1) * Blk<D, N>::HALF + (k * N + j) * Blk<D, N>::NH + (i >> 1);
}

template <typename T, int D>
__device__ __forceinline__ int block_at(const LV<T> &L, int bx, int by, int bz) {
    if (bx < 0 || by < 0 || bx >= L.nb || by >= L.nb) return -2;
    if (D == 3 && (bz < 0 || bz >= L.nb)) return -2;
    return L.lut[D == 3 ? (bz * L.nb + by) * L.nb + bx : by * L.nb + bx];
}

// zero-flux (Neumann) domain face of axis ax, side s: the ghost is the
// inside value (mirror); otherwise Dirichlet, ghost 2 phi_b - inside
__device__ __forceinline__ bool zero_flux(int mask, int ax, int s) { return (mask >> (2 * ax + (s > 0))) & 1; }

template <int D>
__device__ __forceinline__ int face_slot(int ax, int s, int gi, int gj, int gk, int n, int nface) {
    int t;
    if (D == 3) t = ax == 0 ? gk * n + gj : (ax == 1 ? gk * n + gi : gj * n + gi);
    else t = ax == 0 ? gj : gi;
    return (2 * ax + (s > 0)) * nface + t;
}

// value at global cell Q of a level (block edge NB); Q inside the domain
template <typename T, int D, int NB>
__device__ __forceinline__ T level_value(const LV<T> &L, const T *f, int qi, int qj, int qk) {
    const int b = block_at<T, D>(L, qi / NB, qj / NB, D == 3 ? qk / NB : 0);
    if (b < 0) return T(0);  // excluded by 2:1 balance
    return f[(long long)b * Blk<D, NB>::CPB + split_of<D, NB>(qi % NB, qj % NB, D == 3 ? qk % NB : 0)];
}

// refinement-boundary ghost for fine cell G in direction (ax, s)
template <typename T, int D, int N>
__device__ __forceinline__ T cf_ghost(const LV<T> &Lc, const T *phic, int gi, int gj, int gk, int ax, int s, T f1,
                                   T f2) {
    int ng[3] = {gi, gj, gk};
    ng[ax] += s;
    const int C[3] = {ng[0] >> 1, ng[1] >> 1, D == 3 ? ng[2] >> 1 : 0};
    const T Cv = level_value<T, D, N>(Lc, phic, C[0], C[1], C[2]);
    T Ck = Cv;
    for (int t = 0; t < D; t++) {
        if (t == ax) continue;
        const T st = (ng[t] & 1) ? T(1) : T(-1);
        int P[3] = {C[0], C[1], C[2]}, M[3] = {C[0], C[1], C[2]};
        P[t] += 1;
        M[t] -= 1;
        T cp, cm;
        if (P[t] >= Lc.n) {
            T bv = Lc.bcv ? Lc.bcv[face_slot<D>(t, 1, C[0], C[1], C[2], Lc.n, Lc.nface)] : T(0);
            cp = zero_flux(Lc.neumann, t, 1) ? Cv : T(2) * bv - Cv;
        } else {
            cp = level_value<T, D, N>(Lc, phic, P[0], P[1], P[2]);
        }
        if (M[t] < 0) {
            T bv = Lc.bcv ? Lc.bcv[face_slot<D>(t, -1, C[0], C[1], C[2], Lc.n, Lc.nface)] : T(0);
            cm = zero_flux(Lc.neumann, t, -1) ? Cv : T(2) * bv - Cv;
        } else {
            cm = level_value<T, D, N>(Lc, phic, M[0], M[1], M[2]);
        }
        Ck = Ck + st * (cp - cm) / T(8);
    }
    return T(0.5) * Ck + T(0.75) * f1 - T(0.25) * f2;
}

// The 2D neighbour values (ghosts included) of local cell (i,j,k) of block
// `blk`.  `own` is the cell's current value (needed only by ghosts).
template <typename T, int D, int N, bool ZERO>
__device__ __forceinline__ void gather(const LV<T> &L, const LV<T> &Lc, const T *phi, const T *phic,
                                       long long base, const int *snb, int4 P, int i, int j, int k, T own,
                                       T v[2 * D]) {
    int pending = 0;
#pragma unroll
    for (int d = 0; d < 2 * D; d++) {
        const int ax = d >> 1, s = (d & 1) ? 1 : -1;
        int c[3] = {i, j, k};
        c[ax] += s;
        if (ZERO) {
            v[d] = T(0);
            if (c[ax] < 0 || c[ax] >= N) {
                const int nbk = snb[d];
                if (nbk == -2 && !zero_flux(L.neumann, ax, s)) {
                    const int gi = P.x * N + i, gj = P.y * N + j, gk = D == 3 ? P.z * N + k : 0;
                    v[d] = L.bcv ? T(2) * L.bcv[face_slot<D>(ax, s, gi, gj, gk, L.n, L.nface)] : T(0);
                }
            }
            continue;
        }
        if (c[ax] >= 0 && c[ax] < N) {
            v[d] = phi[base + split_of<D, N>(c[0], c[1], c[2])];
        } else {
            const int nbk = snb[d];
            c[ax] = c[ax] < 0 ? N - 1 : 0;
            if (nbk >= 0) {
                v[d] = phi[(long long)nbk * Blk<D, N>::CPB + split_of<D, N>(c[0], c[1], c[2])];
            } else if (nbk == -2) {
                const int gi = P.x * N + i, gj = P.y * N + j, gk = D == 3 ? P.z * N + k : 0;
                const T bv = L.bcv ? L.bcv[face_slot<D>(ax, s, gi, gj, gk, L.n, L.nface)] : T(0);
                v[d] = zero_flux(L.neumann, ax, s) ? own : T(2) * bv - own;
            } else {
                pending |= 1 << d;
                v[d] = T(0);
            }
        }
    }
    if (pending) {
#pragma unroll
        for (int d = 0; d < 2 * D; d++) {
            if (!(pending >> d & 1)) continue;
            const int ax = d >> 1, s = (d & 1) ? 1 : -1;
            const int gi = P.x * N + i, gj = P.y * N + j, gk = D == 3 ? P.z * N + k : 0;
            v[d] = cf_ghost<T, D, N>(Lc, phic, gi, gj, gk, ax, s, own, v[d ^ 1]);
        }
    }
}

template <typename T, int D, int N>
__device__ __forceinline__ bool on_block_face(int i, int j, int k) {
    return i == 0 || i == N - 1 || j == 0 || j == N - 1 || (D == 3 && (k == 0 || k == N - 1));
}

// right-hand side of this workgroup: grid y walks the launch's lane list
// (the running right-hand sides), or all of them when there is none
// |r| for the max-norm reductions, NaN as +Inf (fmax would drop a NaN, so a
// non-finite residual must enter the max as +Inf)
__device__ __forceinline__ double abs_nan_inf(double r) {
    const double a = fabs(r);
    return a == a ? a : __longlong_as_double(0x7ff0000000000000ll);
}

template <typename T>
__device__ __forceinline__ int rhs_of(const LV<T> &L) {
    return L.lanes ? L.lanes[blockIdx.y] : (int)blockIdx.y;
}

// the norm slot of this workgroup for right-hand side rhs
__device__ __forceinline__ unsigned long long *norm_slot(unsigned long long *out, int rhs) {
    return out + ((long long)rhs * kNormSlots + blockIdx.x % kNormSlots) * kNormStride;
}

template <typename T>
__device__ __forceinline__ bool inactive(const LV<T> &L) {
    return L.active && !L.active[rhs_of(L)];
}

template <typename T, int D>
__device__ __forceinline__ void load_neighbours(const LV<T> &L, int4 P, int *snb, int *smo, int b) {
    if ((int)threadIdx.x < 2 * D) {
        const int d = threadIdx.x, ax = d >> 1, s = (d & 1) ? 1 : -1;
        int q[3] = {P.x, P.y, P.z};
        q[ax] += s;
        snb[d] = block_at<T, D>(L, q[0], q[1], q[2]);
    }
    if (threadIdx.x == 0) *smo = L.map_off ? L.map_off[b] : -1;
}

// ------------------------------------------------------ red-black sweep
// One colour of Gauss-Seidel (Sec. 2.2): phi_i <- (g_i - b_i - sum_uncut
// c_ij phi_j) / c_ii, all cells of `color` of the level.
template <typename T, int D, int N>
__global__ __launch_bounds__((Blk<D, N>::THREADS)) void k_gs_half(LV<T> L, LV<T> Lc, int color) {
    if (inactive(L)) return;
    using B = Blk<D, N>;
    const int blk = blockIdx.x;
    __shared__ int snb[2 * D];
    __shared__ int smo;
    const int4 P = L.pos[blk];
    load_neighbours<T, D>(L, P, snb, &smo, blk);
    __syncthreads();
    T *phi = L.phi + (long long)rhs_of(L) * L.fstride;
    const T *g = L.g + (long long)rhs_of(L) * L.fstride;
    const T *phic = Lc.phi ? Lc.phi + (long long)rhs_of(L) * Lc.fstride : nullptr;
    const long long base = (long long)blk * B::CPB;
    const int mo = smo;
    const T inv2d = T(1) / T(2 * D);
    for (int q = threadIdx.x; q < B::HALF; q += B::THREADS) {
        const int h = q % B::NH, j = (q / B::NH) % N, k = D == 3 ? q / (B::NH * N) : 0;
        const int i = 2 * h + ((color + j + k) & 1);
        const long long me = base + color * B::HALF + q;
        const T own = on_block_face<T, D, N>(i, j, k) ? phi[me] : T(0);
        T v[2 * D];
        gather<T, D, N, false>(L, Lc, phi, phic, base, snb, P, i, j, k, own, v);
        const int ri = mo >= 0 ? L.map[mo + color * B::HALF + q] : -1;
        T nv;
        if (ri < 0) {
            T s = v[0];
#pragma unroll
            for (int d = 1; d < 2 * D; d++) s += v[d];
            nv = (s - L.dx2 * g[me]) * inv2d;
        } else {
            const T *r = L.rec + 8 * (long long)ri;
            T s = T(0);
#pragma unroll
            for (int d = 0; d < 2 * D; d++) s += r[d] * v[d];
            const T bt = L.b ? L.b[ri] : T(0);
            nv = (g[me] - bt - s) * r[7];
        }
        phi[me] = nv;
    }
}

// L phi at a cell (Sec. 3.3): sum c_j phi_j + c_ii phi_i + b_i
template <typename T, int D, int N, bool ZERO>
__device__ __forceinline__ T apply_op(const LV<T> &L, const LV<T> &Lc, const T *phi, const T *phic, long long base,
                                      const int *snb, int4 P, int mo, int i, int j, int k, T own) {
    T v[2 * D];
    gather<T, D, N, ZERO>(L, Lc, phi, phic, base, snb, P, i, j, k, own, v);
    const int si = split_of<D, N>(i, j, k);
    const int ri = mo >= 0 ? L.map[mo + si] : -1;
    if (ri < 0) {
        T s = v[0];
#pragma unroll
        for (int d = 1; d < 2 * D; d++) s += v[d];
        return L.inv_dx2 * (s - T(2 * D) * own);
    }
    const T *r = L.rec + 8 * (long long)ri;
    T s = T(0);
#pragma unroll
    for (int d = 0; d < 2 * D; d++) s += r[d] * v[d];
    const T bt = L.b ? L.b[ri] : T(0);
    return s + r[6] * own + bt;
}

// ------------------------------------------------------- restriction
// FAS restriction (Sec. 2.2): phi_c = mean of the 2^D children, and the
// coarse g holds the mean of the children's residuals until k_fas_rhs adds
// L_c phi_c.  One workgroup per fine block; thread per coarse cell.
template <typename T, int D, int N, int NC>
__global__ __launch_bounds__(256) void k_restrict_fas(LV<T> L, LV<T> Lc, int into_old) {
    if (inactive(L)) return;
    constexpr int H = N / 2, NCELL = D == 3 ? H * H * H : H * H;
    const int blk = blockIdx.x;
    __shared__ int snb[2 * D];
    __shared__ int smo;
    const int4 P = L.pos[blk];
    load_neighbours<T, D>(L, P, snb, &smo, blk);
    __syncthreads();
    const T *phi = L.phi + (long long)rhs_of(L) * L.fstride;
    const T *g = L.g + (long long)rhs_of(L) * L.fstride;
    const T *phic = Lc.phi + (long long)rhs_of(L) * Lc.fstride;
    T *phiw = (into_old ? Lc.old : Lc.phi) + (long long)rhs_of(L) * Lc.fstride;
    T *gw = Lc.g + (long long)rhs_of(L) * Lc.fstride;
    const long long base = (long long)blk * Blk<D, N>::CPB;
    const int C0[3] = {P.x * H, P.y * H, D == 3 ? P.z * H : 0};
    const int pb = block_at<T, D>(Lc, C0[0] / NC, C0[1] / NC, D == 3 ? C0[2] / NC : 0);
    if (pb < 0) return;
    const T inv = T(1) / T(1 << D);
    for (int c = threadIdx.x; c < NCELL; c += blockDim.x) {
        const int ci = c % H, cj = (c / H) % H, ck = D == 3 ? c / (H * H) : 0;
        T sp = T(0), sr = T(0);
#pragma unroll
        for (int ch = 0; ch < (1 << D); ch++) {
            const int i = 2 * ci + (ch & 1), j = 2 * cj + ((ch >> 1) & 1), k = D == 3 ? 2 * ck + ((ch >> 2) & 1) : 0;
            const T own = phi[base + split_of<D, N>(i, j, k)];
            const T lphi = apply_op<T, D, N, false>(L, Lc, phi, phic, base, snb, P, smo, i, j, k, own);
            sp += own;
            sr += g[base + split_of<D, N>(i, j, k)] - lphi;
        }
        const int gi = C0[0] + ci, gj = C0[1] + cj, gk = C0[2] + ck;
        const long long o = (long long)pb * Blk<D, NC>::CPB + split_of<D, NC>(gi % NC, gj % NC, D == 3 ? gk % NC : 0);
        phiw[o] = sp * inv;
        gw[o] = sr * inv;
    }
}

template <typename T, int D, int N>
__global__ __launch_bounds__(256) void k_copy_parents(LV<T> L, int leaves_only) {
    if (inactive(L)) return;
    const int blk = blockIdx.x;
    const long long o = (long long)rhs_of(L) * L.fstride + (long long)blk * Blk<D, N>::CPB;
    if (L.leaf[blk]) {
        for (int c = threadIdx.x; c < Blk<D, N>::CPB; c += blockDim.x) L.old[o + c] = L.phi[o + c];
        return;
    }
    if (leaves_only) return;
    for (int c = threadIdx.x; c < Blk<D, N>::CPB; c += blockDim.x) L.phi[o + c] = L.old[o + c];
}

// restriction of the rhs for a first FMG without initial guess
template <typename T, int D, int N, int NC>
__global__ __launch_bounds__(256) void k_restrict_rhs(LV<T> L, LV<T> Lc) {
    if (inactive(L)) return;
    constexpr int H = N / 2, NCELL = D == 3 ? H * H * H : H * H;
    const int blk = blockIdx.x;
    const int4 P = L.pos[blk];
    const T *g = L.g + (long long)rhs_of(L) * L.fstride;
    T *gw = Lc.g + (long long)rhs_of(L) * Lc.fstride;
    const long long base = (long long)blk * Blk<D, N>::CPB;
    const int C0[3] = {P.x * H, P.y * H, D == 3 ? P.z * H : 0};
    const int pb = block_at<T, D>(Lc, C0[0] / NC, C0[1] / NC, D == 3 ? C0[2] / NC : 0);
    if (pb < 0) return;
    const T inv = T(1) / T(1 << D);
    for (int c = threadIdx.x; c < NCELL; c += blockDim.x) {
        const int ci = c % H, cj = (c / H) % H, ck = D == 3 ? c / (H * H) : 0;
        T s = T(0);
#pragma unroll
        for (int ch = 0; ch < (1 << D); ch++) {
            const int i = 2 * ci + (ch & 1), j = 2 * cj + ((ch >> 1) & 1), k = D == 3 ? 2 * ck + ((ch >> 2) & 1) : 0;
            s += g[base + split_of<D, N>(i, j, k)];
        }
        const int gi = C0[0] + ci, gj = C0[1] + cj, gk = C0[2] + ck;
        gw[(long long)pb * Blk<D, NC>::CPB + split_of<D, NC>(gi % NC, gj % NC, D == 3 ? gk % NC : 0)] = s * inv;
    }
}

// phi_c = mean of children only (composite-grid synchronisation)
template <typename T, int D, int N, int NC>
__global__ __launch_bounds__(256) void k_restrict_phi(LV<T> L, LV<T> Lc) {
    if (inactive(L)) return;
    constexpr int H = N / 2, NCELL = D == 3 ? H * H * H : H * H;
    const int blk = blockIdx.x;
    const int4 P = L.pos[blk];
    const T *phi = L.phi + (long long)rhs_of(L) * L.fstride;
    T *pw = Lc.phi + (long long)rhs_of(L) * Lc.fstride;
    const long long base = (long long)blk * Blk<D, N>::CPB;
    const int C0[3] = {P.x * H, P.y * H, D == 3 ? P.z * H : 0};
    const int pb = block_at<T, D>(Lc, C0[0] / NC, C0[1] / NC, D == 3 ? C0[2] / NC : 0);
    if (pb < 0) return;
    const T inv = T(1) / T(1 << D);
    for (int c = threadIdx.x; c < NCELL; c += blockDim.x) {
        const int ci = c % H, cj = (c / H) % H, ck = D == 3 ? c / (H * H) : 0;
        T s = T(0);
#pragma unroll
        for (int ch = 0; ch < (1 << D); ch++) {
            const int i = 2 * ci + (ch & 1), j = 2 * cj + ((ch >> 1) & 1), k = D == 3 ? 2 * ck + ((ch >> 2) & 1) : 0;
            s += phi[base + split_of<D, N>(i, j, k)];
        }
        const int gi = C0[0] + ci, gj = C0[1] + cj, gk = C0[2] + ck;
        pw[(long long)pb * Blk<D, NC>::CPB + split_of<D, NC>(gi % NC, gj % NC, D == 3 ? gk % NC : 0)] = s * inv;
    }
}

// FAS right-hand side on parent blocks: g = L phi + (restricted residual);
// old = phi on every block of the level.  Coarse ghosts must be current,
// hence a launch of its own after the restriction.
template <typename T, int D, int N>
__global__ __launch_bounds__((Blk<D, N>::THREADS)) void k_fas_rhs(LV<T> L, LV<T> Lc, int do_rhs) {
    if (inactive(L)) return;
    using B = Blk<D, N>;
    const int blk = blockIdx.x;
    __shared__ int snb[2 * D];
    __shared__ int smo;
    const int4 P = L.pos[blk];
    load_neighbours<T, D>(L, P, snb, &smo, blk);
    __syncthreads();
    T *phi = L.phi + (long long)rhs_of(L) * L.fstride;
    T *g = L.g + (long long)rhs_of(L) * L.fstride;
    T *old = L.old + (long long)rhs_of(L) * L.fstride;
    const T *phic = Lc.phi ? Lc.phi + (long long)rhs_of(L) * Lc.fstride : nullptr;
    const long long base = (long long)blk * B::CPB;
    const bool parent = !L.leaf[blk];
    for (int c = threadIdx.x; c < B::CPB; c += B::THREADS) {
        const int i = c % N, j = (c / N) % N, k = D == 3 ? c / (N * N) : 0;
        const long long me = base + split_of<D, N>(i, j, k);
        const T own = phi[me];
        if (parent && do_rhs) {
            const T lphi = apply_op<T, D, N, false>(L, Lc, phi, phic, base, snb, P, smo, i, j, k, own);
            g[me] = lphi + g[me];
        }
        old[me] = own;
    }
}

// ------------------------------------------------------ prolongation
// phi_f += sum over the 2^D nearest coarse cells of prod_a (3/4 | 1/4) e_c,
// e_c = phi_c - old_c (Sec. 2.2, 3.4); outside the domain e_c is reflected
// with a sign flip per axis.  Solution mode (first FMG without guess): e_c =
// phi_c with Dirichlet ghosts, linear extrapolation at edges/corners.
// Coarse solution value at coarse cell q for the first interpolation of a
// nested iteration, with ghosts outside the domain: across the first
// outside axis the mirror cell (zero-flux face), else 2 phi_b - inside when
// only that axis is outside, else linear extrapolation 2 v(q - s e) -
// v(q - 2 s e).  Each step brings one axis inside, so DEPTH = D + 1 levels
// of expansion always suffice.
template <typename T, int D, int NC, int DEPTH>
__device__ __forceinline__ T coarse_sol(const LV<T> &Lc, const T *phic, int q0, int q1, int q2) {
    const int q[3] = {q0, q1, q2};
    int out = -1, nout = 0;
    for (int a = 0; a < D; a++)
        if (q[a] < 0 || q[a] >= Lc.n) {
            nout++;
            if (out < 0) out = a;
        }
    if (nout == 0 || DEPTH == 0) return level_value<T, D, NC>(Lc, phic, q[0], q[1], q[2]);
    const int s = q[out] < 0 ? -1 : 1;
    int a1[3] = {q[0], q[1], q[2]};
    a1[out] -= s;
    if (zero_flux(Lc.neumann, out, s)) return coarse_sol<T, D, NC, (DEPTH > 0 ? DEPTH - 1 : 0)>(Lc, phic, a1[0], a1[1], a1[2]);
    if (nout == 1) {
        const T bv = Lc.bcv ? Lc.bcv[face_slot<D>(out, s, a1[0], a1[1], a1[2], Lc.n, Lc.nface)] : T(0);
        return T(2) * bv - level_value<T, D, NC>(Lc, phic, a1[0], a1[1], a1[2]);
    }
    int a2[3] = {q[0], q[1], q[2]};
    a2[out] -= 2 * s;
    return T(2) * coarse_sol<T, D, NC, (DEPTH > 0 ? DEPTH - 1 : 0)>(Lc, phic, a1[0], a1[1], a1[2]) -
           coarse_sol<T, D, NC, (DEPTH > 0 ? DEPTH - 1 : 0)>(Lc, phic, a2[0], a2[1], a2[2]);
}

// Coarse correction e = phi_c - old_c at coarse cell q for the
// prolongation; outside the domain it is mirrored, with a sign flip per
// Dirichlet axis (homogeneous ghost -e) and none per zero-flux axis.  In
// solution mode the coarse solution with its ghosts (coarse_sol).
template <typename T, int D, int NC, bool SOL>
__device__ __forceinline__ T coarse_e(const LV<T> &Lc, const T *phic, const T *oldc, int x0, int x1, int x2) {
    if (SOL) return coarse_sol<T, D, NC, D + 1>(Lc, phic, x0, x1, x2);
    int q[3] = {x0, x1, x2};
    T sign = T(1);
    for (int a = 0; a < D; a++) {
        if (q[a] < 0) {
            q[a] = 0;
            if (!zero_flux(Lc.neumann, a, -1)) sign = -sign;
        } else if (q[a] >= Lc.n) {
            q[a] = Lc.n - 1;
            if (!zero_flux(Lc.neumann, a, 1)) sign = -sign;
        }
    }
    const int b = block_at<T, D>(Lc, q[0] / NC, q[1] / NC, D == 3 ? q[2] / NC : 0);
    if (b < 0) return T(0);
    const long long o = (long long)b * Blk<D, NC>::CPB + split_of<D, NC>(q[0] % NC, q[1] % NC, D == 3 ? q[2] % NC : 0);
    return sign * (phic[o] - oldc[o]);
}

template <typename T, int D, int N, int NC>
__global__ __launch_bounds__(256) void k_prolong(LV<T> L, LV<T> Lc, int solution) {
    if (inactive(L)) return;
    constexpr int H = N / 2, NCELL = D == 3 ? H * H * H : H * H;
    const int blk = blockIdx.x;
    const int4 P = L.pos[blk];
    T *phi = L.phi + (long long)rhs_of(L) * L.fstride;
    const T *phic = Lc.phi + (long long)rhs_of(L) * Lc.fstride;
    const T *oldc = Lc.old + (long long)rhs_of(L) * Lc.fstride;
    const long long base = (long long)blk * Blk<D, N>::CPB;
    const int C0[3] = {P.x * H, P.y * H, D == 3 ? P.z * H : 0};
    for (int c = threadIdx.x; c < NCELL; c += blockDim.x) {
        const int ci = c % H, cj = (c / H) % H, ck = D == 3 ? c / (H * H) : 0;
        const int G[3] = {C0[0] + ci, C0[1] + cj, C0[2] + ck};
        T E[D == 3 ? 27 : 9];
#pragma unroll
        for (int z = 0; z < (D == 3 ? 3 : 1); z++)
#pragma unroll
            for (int y = 0; y < 3; y++)
#pragma unroll
                for (int x = 0; x < 3; x++)
                    E[(z * 3 + y) * 3 + x] =
                        solution ? coarse_e<T, D, NC, true>(Lc, phic, oldc, G[0] + x - 1, G[1] + y - 1, D == 3 ? G[2] + z - 1 : 0)
                                 : coarse_e<T, D, NC, false>(Lc, phic, oldc, G[0] + x - 1, G[1] + y - 1, D == 3 ? G[2] + z - 1 : 0);
#pragma unroll
        for (int ch = 0; ch < (1 << D); ch++) {
            const int a = ch & 1, bb = (ch >> 1) & 1, cc = (ch >> 2) & 1;
            const int o[3] = {a ? 1 : -1, bb ? 1 : -1, cc ? 1 : -1};
            T e = T(0);
#pragma unroll
            for (int dl = 0; dl < (1 << D); dl++) {
                T w = T(1);
                int idx[3] = {1, 1, 1};
#pragma unroll
                for (int ax = 0; ax < D; ax++) {
                    const int on = (dl >> ax) & 1;
                    w = w * (on ? T(0.25) : T(0.75));
                    if (on) idx[ax] += o[ax];
                }
                e = e + w * E[((D == 3 ? idx[2] : 0) * 3 + idx[1]) * 3 + idx[0]];
            }
            const int i = 2 * ci + a, j = 2 * cj + bb, k = D == 3 ? 2 * ck + cc : 0;
            phi[base + split_of<D, N>(i, j, k)] += e;
        }
    }
}

// ------------------------------------------------------ coarse solve
// Exact solve on the single-block coarsest grid (8^D cells): rhs_i = S_i (g_i
// - b_i - sum over uncut domain links 2 c phi_b), phi = M rhs, where M is the
// inverse of the row-equilibrated operator.  Grid: x = row tiles, y = rhs.
template <typename T, int D, bool FAS>
__global__ __launch_bounds__(256) void k_coarse_solve(LV<T> L0, const double *M, const double *S) {
    if (inactive(L0)) return;
    constexpr int NB = 8, NCELL = D == 3 ? 512 : 64;
    constexpr int ROWS_PER_WG = D == 3 ? 8 : 16, RPW = ROWS_PER_WG / 4, CPL = NCELL / 64;
    __shared__ double rhs[NCELL];
    // the wave's rows of the inverse do not depend on the rhs: their loads
    // are issued first and complete while the rhs vector is formed
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    double mrow[RPW][CPL];
#pragma unroll
    for (int r = 0; r < RPW; r++)
#pragma unroll
        for (int c = 0; c < CPL; c++)
            mrow[r][c] = M[(long long)(blockIdx.x * ROWS_PER_WG + wave + 4 * r) * NCELL + lane + 64 * c];
    const T *g = L0.g + (long long)rhs_of(L0) * L0.fstride;
    T *phi = L0.phi + (long long)rhs_of(L0) * L0.fstride;
    const int mo = L0.map_off ? L0.map_off[0] : -1;
    const double inv = 1.0 / ((double)L0.dx2);
    for (int c = threadIdx.x; c < NCELL; c += blockDim.x) {
        const int i = c % NB, j = (c / NB) % NB, k = D == 3 ? c / (NB * NB) : 0;
        const int si = split_of<D, NB>(i, j, k);
        const int ri = mo >= 0 ? L0.map[mo + si] : -1;
        double r;
        if (FAS) {
            // FAS right-hand side of the coarsest level, g + L phi with phi
            // the restricted values in old (the arithmetic of k_fas_rhs3)
            const T *old = L0.old + (long long)rhs_of(L0) * L0.fstride;
            const T own = old[si];
            T v[6];
#pragma unroll
            for (int d = 0; d < 6; d++) {
                const int ax = d >> 1, sg = (d & 1) ? 1 : -1;
                int q[3] = {i, j, k};
                q[ax] += sg;
                if (q[ax] >= 0 && q[ax] < NB) {
                    v[d] = old[split_of<D, NB>(q[0], q[1], q[2])];
                } else {
                    const T bv = L0.bcv ? L0.bcv[face_slot<D>(ax, sg, i, j, k, NB, L0.nface)] : T(0);
                    v[d] = zero_flux(L0.neumann, ax, sg) ? own : T(2) * bv - own;
                }
            }
            T lp;
            if (ri < 0) {
                lp = L0.inv_dx2 * ((((v[0] + v[1]) + (v[2] + v[3])) + (v[4] + v[5])) - T(6) * own);
            } else {
                const T *rr = L0.rec + 8 * (long long)ri;
                T sm = T(0);
#pragma unroll
                for (int d = 0; d < 6; d++) sm += rr[d] * v[d];
                lp = sm + rr[6] * own + (L0.b ? L0.b[ri] : T(0));
            }
            r = (double)(lp + g[si]);
        } else {
            r = (double)g[si];
        }
        if (ri >= 0 && L0.b) r -= (double)L0.b[ri];
        for (int d = 0; d < 2 * D; d++) {
            const int ax = d >> 1, s = (d & 1) ? 1 : -1;
            int q[3] = {i, j, k};
            q[ax] += s;
            if (q[ax] >= 0 && q[ax] < NB) continue;
            const double cc = ri >= 0 ? (double)L0.rec[8 * (long long)ri + d] : inv;
            if (cc == 0.0 || zero_flux(L0.neumann, ax, s)) continue;  // zero flux: folded into the operator
            const double bv = L0.bcv ? (double)L0.bcv[face_slot<D>(ax, s, i, j, k, NB, L0.nface)] : 0.0;
            r -= 2.0 * cc * bv;
        }
        rhs[c] = S[c] * r;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RPW; r++) {
        const int row = blockIdx.x * ROWS_PER_WG + wave + 4 * r;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < CPL; c++) acc += mrow[r][c] * rhs[lane + 64 * c];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lane == 0) {
            const int i = row % NB, j = (row / NB) % NB, k = D == 3 ? row / (NB * NB) : 0;
            phi[split_of<D, NB>(i, j, k)] = (T)acc;
        }
    }
}

// ------------------------------------------------------ residual norm
template <typename T, int D, int N, bool ZERO>
__global__ __launch_bounds__((Blk<D, N>::THREADS)) void k_residual_max(LV<T> L, LV<T> Lc, unsigned long long *out) {
    if (inactive(L)) return;
    using B = Blk<D, N>;
    const int blk = blockIdx.x;
    __shared__ int snb[2 * D];
    __shared__ int smo;
    __shared__ double wmax[B::THREADS / 64 + 1];
    if (!L.leaf[blk]) return;
    const int4 P = L.pos[blk];
    load_neighbours<T, D>(L, P, snb, &smo, blk);
    __syncthreads();
    const T *phi = L.phi + (long long)rhs_of(L) * L.fstride;
    const T *g = L.g + (long long)rhs_of(L) * L.fstride;
    const T *phic = Lc.phi ? Lc.phi + (long long)rhs_of(L) * Lc.fstride : nullptr;
    const long long base = (long long)blk * B::CPB;
    double m = 0.0;
    for (int c = threadIdx.x; c < B::CPB; c += B::THREADS) {
        const int i = c % N, j = (c / N) % N, k = D == 3 ? c / (N * N) : 0;
        const long long me = base + split_of<D, N>(i, j, k);
        const T own = ZERO ? T(0) : phi[me];
        const T lphi = apply_op<T, D, N, ZERO>(L, Lc, phi, phic, base, snb, P, smo, i, j, k, own);
        m = fmax(m, abs_nan_inf((double)(g[me] - lphi)));
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if (threadIdx.x % 64 == 0) wmax[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(B::THREADS + 63) / 64; w++) m = fmax(m, wmax[w]);
        if (m != m) m = __longlong_as_double(0x7ff0000000000000ll);  // NaN -> +Inf
        atomicMax(norm_slot(out, rhs_of(L)), (unsigned long long)__double_as_longlong(m));
    }
}

// ------------------------------------------------------ data movement
template <int D, int N>
__global__ void k_scatter_leaf(LV<double> L, const int *lb, const double *src, long long sstride, long long base,
                               int field) {
    using B = Blk<D, N>;
    const int blk = lb[blockIdx.x];
    double *dst = (field == 0 ? L.phi : L.g) + (long long)blockIdx.y * L.fstride + (long long)blk * B::CPB;
    const double *s = src + (long long)blockIdx.y * sstride + base + (long long)blockIdx.x * B::CPB;
    for (int c = threadIdx.x; c < B::CPB; c += blockDim.x) {
        const int i = c % N, j = (c / N) % N, k = D == 3 ? c / (N * N) : 0;
        dst[split_of<D, N>(i, j, k)] = s[c];
    }
}

template <int D, int N>
__global__ void k_gather_leaf(LV<double> L, const int *lb, double *dst, long long dstride, long long base) {
    using B = Blk<D, N>;
    const int blk = lb[blockIdx.x];
    const double *src = L.phi + (long long)blockIdx.y * L.fstride + (long long)blk * B::CPB;
    double *d = dst + (long long)blockIdx.y * dstride + base + (long long)blockIdx.x * B::CPB;
    for (int c = threadIdx.x; c < B::CPB; c += blockDim.x) {
        const int i = c % N, j = (c / N) % N, k = D == 3 ? c / (N * N) : 0;
        d[c] = src[split_of<D, N>(i, j, k)];
    }
}

// grad phi of the leaf cells of one level (Sec. 4.3, the application's
// field): on every face the difference to the neighbour value or ghost over
// dx, or (phi_b - phi_i)/(d dx) towards a boundary on that link; each
// component is the mean of its two faces.  Post-processing, run once per
// solution: one thread per cell, no LDS staging.
template <int D, int N>
__global__ void k_gradient(LV<double> L, LV<double> Lc, const int *lb, const int *meta, const double *d6,
                           const int *inside, const double *pb, int inside_zero, double *out, long long ostride,
                           long long base) {
    using B = Blk<D, N>;
    const int blk = lb[blockIdx.x];
    __shared__ int snb[2 * D];
    __shared__ int smo;
    const int4 P = L.pos[blk];
    load_neighbours<double, D>(L, P, snb, &smo, blk);
    __syncthreads();
    const double *phi = L.phi + (long long)blockIdx.y * L.fstride;
    const double *phic = Lc.phi ? Lc.phi + (long long)blockIdx.y * Lc.fstride : nullptr;
    const double *pbr = pb;
    const long long bb = (long long)blk * B::CPB;
    double *o = out + (long long)blockIdx.y * ostride + 3 * (base + (long long)blockIdx.x * B::CPB);
    const double inv = 1.0 / sqrt(L.dx2);
    for (int c = threadIdx.x; c < B::CPB; c += blockDim.x) {
        const int i = c % N, j = (c / N) % N, k = D == 3 ? c / (N * N) : 0;
        const int si = split_of<D, N>(i, j, k);
        const double own = phi[bb + si];
        const int ri = smo >= 0 ? L.map[smo + si] : -1;
        const int cut = ri >= 0 ? meta[4 * ri + 2] : 0;
        double gr[3] = {0.0, 0.0, 0.0};
        if (!(inside_zero && ri >= 0 && inside[ri])) {
            double v[2 * D];
            gather<double, D, N, false>(L, Lc, phi, phic, bb, snb, P, i, j, k, own, v);
            int pt = ri >= 0 ? meta[4 * ri + 3] : 0;  // points of the cut links, in link order
            for (int ax = 0; ax < D; ax++) {
                double face[2];
                for (int side = 0; side < 2; side++) {
                    const int kk = 2 * ax + side;
                    double dv;
                    if (cut >> kk & 1) dv = (pbr[pt++] - own) / (d6[6 * ri + kk] * sqrt(L.dx2));
                    else dv = (v[kk] - own) * inv;
                    face[side] = side ? dv : -dv;
                }
                gr[ax] = 0.5 * (face[0] + face[1]);
            }
        }
        for (int a = 0; a < 3; a++) o[3 * c + a] = gr[a];
    }
}

// colour-split index for a block edge known only at run time
__device__ __forceinline__ int split_rt(int D, int Nb, int i, int j, int k) {
    const int cpb = D == 3 ? Nb * Nb * Nb : Nb * Nb;
    return ((i + j + k) & 1) * (cpb / 2) + (k * Nb + j) * (Nb / 2) + (i >> 1);
}

// value of the old tree at level lv, global cell (x, y, z) (block must exist)
__device__ __forceinline__ double old_value(int D, const LV<double> &L, int Nb, int b, int rhs, int x, int y, int z) {
    const int cpb = D == 3 ? Nb * Nb * Nb : Nb * Nb;
    return L.phi[(long long)rhs * L.fstride + (long long)b * cpb + split_rt(D, Nb, x % Nb, y % Nb, D == 3 ? z % Nb : 0)];
}

// phi of one level of an adapted tree from the previous tree (whose parent
// cells hold the means of their children): the same cell where the old tree
// has it; one level finer than the old tree: the cell-centred (3/4, 1/4)
// interpolation of the old cells (a neighbour the old level lacks, or one
// outside the domain, is replaced by the centre cell); deeper: the value of
// the old cell containing the centre.
template <int D, int N>
__global__ void k_remap(LV<double> Ln, int il, const LV<double> *Lold, const int *nb_old, const int *lb) {
    using B = Blk<D, N>;
    const int blk = lb[blockIdx.x], rhs = blockIdx.y;
    const int4 P = Ln.pos[blk];
    double *dst = Ln.phi + (long long)rhs * Ln.fstride + (long long)blk * B::CPB;
    for (int c = threadIdx.x; c < B::CPB; c += blockDim.x) {
        const int i = c % N, j = (c / N) % N, k = D == 3 ? c / (N * N) : 0;
        const int g[3] = {P.x * N + i, P.y * N + j, D == 3 ? P.z * N + k : 0};
        const LV<double> &Ls = Lold[il];
        int b = block_at<double, D>(Ls, g[0] / N, g[1] / N, D == 3 ? g[2] / N : 0);
        double val;
        if (b >= 0) {
            val = old_value(D, Ls, N, b, rhs, g[0], g[1], g[2]);
        } else {
            int lv = il - 1, ga[3] = {g[0] >> 1, g[1] >> 1, g[2] >> 1};
            for (; lv > 0; lv--) {
                const int nb = nb_old[lv];
                b = block_at<double, D>(Lold[lv], ga[0] / nb, ga[1] / nb, D == 3 ? ga[2] / nb : 0);
                if (b >= 0) break;
                for (int a = 0; a < 3; a++) ga[a] >>= 1;
            }
            const LV<double> &La = Lold[lv];
            const int nb = nb_old[lv];
            if (lv == 0) b = 0;
            const double ctr = old_value(D, La, nb, b, rhs, ga[0], ga[1], ga[2]);
            if (lv != il - 1) {
                val = ctr;
            } else {
                val = 0.0;
                for (int m = 0; m < (1 << D); m++) {
                    int q[3] = {ga[0], ga[1], ga[2]};
                    double w = 1.0;
                    for (int a = 0; a < D; a++) {
                        const bool far = (m >> a) & 1;
                        w *= far ? 0.25 : 0.75;
                        if (far) q[a] += (g[a] & 1) ? 1 : -1;
                    }
                    double v = ctr;
                    bool inside = true;
                    for (int a = 0; a < D; a++) inside = inside && q[a] >= 0 && q[a] < La.n;
                    if (inside) {
                        const int bq = block_at<double, D>(La, q[0] / nb, q[1] / nb, D == 3 ? q[2] / nb : 0);
                        if (bq >= 0) v = old_value(D, La, nb, bq, rhs, q[0], q[1], q[2]);
                    }
                    val += w * v;
                }
            }
        }
        dst[split_of<D, N>(i, j, k)] = val;
    }
}

template <int D, int N>
__global__ void k_level_copy(double *split, double *canon, int to_split) {
    using B = Blk<D, N>;
    const long long base = (long long)blockIdx.x * B::CPB;
    for (int c = threadIdx.x; c < B::CPB; c += blockDim.x) {
        const int i = c % N, j = (c / N) % N, k = D == 3 ? c / (N * N) : 0;
        if (to_split) split[base + split_of<D, N>(i, j, k)] = canon[base + c];
        else canon[base + c] = split[base + split_of<D, N>(i, j, k)];
    }
}

// mixed precision: FP64 defect on leaf blocks -> FP32 rhs, FP32 phi = 0
template <int D, int N>
__global__ __launch_bounds__((Blk<D, N>::THREADS)) void k_defect(LV<double> L, LV<double> Lc, LV<float> L32,
                                                                const int *lb, unsigned long long *out) {
    if (inactive(L)) return;
    using B = Blk<D, N>;
    const int blk = lb[blockIdx.x];
    __shared__ int snb[2 * D];
    __shared__ int smo;
    __shared__ double wmax[B::THREADS / 64 + 1];
    const int4 P = L.pos[blk];
    load_neighbours<double, D>(L, P, snb, &smo, blk);
    __syncthreads();
    const double *phi = L.phi + (long long)rhs_of(L) * L.fstride;
    const double *g = L.g + (long long)rhs_of(L) * L.fstride;
    const double *phic = Lc.phi ? Lc.phi + (long long)rhs_of(L) * Lc.fstride : nullptr;
    float *g32 = L32.g + (long long)rhs_of(L) * L32.fstride;
    float *p32 = L32.phi + (long long)rhs_of(L) * L32.fstride;
    const long long base = (long long)blk * B::CPB;
    double m = 0.0;
    for (int c = threadIdx.x; c < B::CPB; c += B::THREADS) {
        const int i = c % N, j = (c / N) % N, k = D == 3 ? c / (N * N) : 0;
        const long long me = base + split_of<D, N>(i, j, k);
        const double own = phi[me];
        const double r = g[me] - apply_op<double, D, N, false>(L, Lc, phi, phic, base, snb, P, smo, i, j, k, own);
        m = fmax(m, abs_nan_inf(r));
        g32[me] = (float)r;
        p32[me] = 0.0f;
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if (threadIdx.x % 64 == 0) wmax[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(B::THREADS + 63) / 64; w++) m = fmax(m, wmax[w]);
        if (m != m) m = __longlong_as_double(0x7ff0000000000000ll);
        atomicMax(norm_slot(out, rhs_of(L)), (unsigned long long)__double_as_longlong(m));
    }
}

template <int D, int N>
__global__ void k_update(LV<double> L, LV<float> L32, const int *lb) {
    if (inactive(L)) return;
    using B = Blk<D, N>;
    const int blk = lb[blockIdx.x];
    double *phi = L.phi + (long long)rhs_of(L) * L.fstride + (long long)blk * B::CPB;
    const float *e = L32.phi + (long long)rhs_of(L) * L32.fstride + (long long)blk * B::CPB;
    for (int c = threadIdx.x; c < B::CPB; c += blockDim.x) phi[c] += (double)e[c];
}

__global__ void k_boundary_terms(int D, const int *meta, const double *cfull, int nrec, const double *vals,
                                 double *b64, float *b32) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    const int cut = meta[4 * r + 2];
    int p = meta[4 * r + 3];
    double b = 0.0;
    for (int k = 0; k < 2 * D; k++) {
        if (!(cut >> k & 1)) continue;
        b = b + cfull[6 * r + k] * (vals ? vals[p] : 0.0);
        p++;
    }
    b64[r] = b;
    if (b32) b32[r] = (float)b;
}

__global__ void k_fill(double *p, long long n, double v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fillf(float *p, long long n, float v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(unsigned long long *p, long long n, unsigned long long v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_norm_reduce(unsigned long long *slots, unsigned long long *norm, unsigned long long *mapped,
                              int nrhs) {
    for (int r = threadIdx.x; r < nrhs; r += blockDim.x) {
        unsigned long long m = 0;
        for (int k = 0; k < kNormSlots; k++) {
            unsigned long long *p = slots + ((long long)r * kNormSlots + k) * kNormStride;
            const unsigned long long v = *p;
            m = v > m ? v : m;
            *p = 0;
        }
        norm[r] = m;
        mapped[r] = m;
    }
}
// cycle number cbase + c of a graph solve: record each running rhs's norm,
// stop it when converged, non-finite, or at the last of max_cycles cycles;
// the last launch of a chunk of `advance` cycles moves cbase on by it
__global__ void k_converge(const unsigned long long *norm, const double *thresh, int *active, double *hist, int c,
                           int nrhs, int *cbase, int max_cycles, int advance) {
    const int cc = c + *cbase;
    if (cc < max_cycles)
        for (int r = threadIdx.x; r < nrhs; r += blockDim.x) {
            if (!active[r]) continue;
            const double v = __longlong_as_double((long long)norm[r]);
            hist[(long long)cc * nrhs + r] = v;
            if (v <= thresh[r] || !(v == v) || cc + 1 >= max_cycles) active[r] = 0;
        }
    __syncthreads();
    if (advance && threadIdx.x == 0) *cbase = cc - c + advance;
}
__global__ void k_copy_d2f(const double *s, float *d, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        d[i] = (float)s[i];
}
__global__ void k_copy_f2d(const float *s, double *d, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        d[i] = (double)s[i];
}
__global__ void k_check_finite(const double *p, long long n, int *flag) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        if (!isfinite(p[i])) atomicOr(flag, 1);
}

// ============================================================ 3D, LDS-staged
// For 3D levels every per-level operation works colour by colour: the other
// colour of the block, plus a one-cell halo from the face neighbours, is
// staged in LDS (26 KB in FP64 for 16^3 blocks), while the cell's own
// values, g and record-map entries are prefetched into registers, so that
// every HBM load of a workgroup is in flight before the first LDS barrier.
// Ghost values at domain faces and refinement boundaries are formed per
// cell as in gather().  Workgroup w runs on XCD w mod 8; blocks are mapped
// so that each XCD walks a contiguous Morton range of the level, which
// keeps face halos in that XCD's L2.

__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
    const int q = nb >> 3, r = nb & 7;
    return xcd * q + min(xcd, r) + slot;
}

// Order 2, for a complete level of nb^3 blocks (nb a power of two >= 2):
// XCD x takes Morton octant x (an (nb/2)^3 cube, a contiguous index range)
// and walks it x-fastest, so the face neighbours inside the octant are at
// most (nb/2)^2 workgroups apart in its dispatch order and their halos are
// read while still in that XCD's L2.  Block index = Morton code with x in
// bit 0, y in bit 1, z in bit 2 of each triple (the tree's order).
__device__ __forceinline__ int spread3(int v) {
    int r = 0;
#pragma unroll
    for (int b = 0; b < 10; b++) r |= ((v >> b) & 1) << (3 * b);
    return r;
}
__device__ __forceinline__ int octant_block(int nb) {
    const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3, h = nb >> 1;
    const int i = slot % h, j = (slot / h) % h, k = slot / (h * h);
    return xcd * h * h * h + (spread3(i) | (spread3(j) << 1) | (spread3(k) << 2));
}

// block of this workgroup: order 0 maps XCD-contiguous Morton ranges as
// above, order 1 keeps the hardware order (consecutive blocks on
// consecutive XCDs), order 2 the octant walk (complete levels; otherwise
// order 0); the result of every block is the same either way
template <typename T>
__device__ __forceinline__ int block_of(const LV<T> &L) {
    if (L.order == 1) return (int)blockIdx.x;
    if (L.order == 2 && L.nb >= 2 && (L.nb & (L.nb - 1)) == 0 && L.nblocks == L.nb * L.nb * L.nb)
        return octant_block(L.nb);
    return xcd_block();
}

// position in a leaf-block list of this workgroup (a launch over the list):
// the list holds the level's leaf blocks in Morton order, so the same
// XCD-contiguous ranges as block_of keep face halos in one XCD's L2
template <typename T>
__device__ __forceinline__ int leaf_slot(const LV<T> &L) {
    return L.order == 1 ? (int)blockIdx.x : xcd_block();
}

// one colour of a block with halo: (N+2) x (N+2) x (N/2+2), index (k, j, h)
template <int N>
struct ColTile {
    static constexpr int NH = N / 2, HX = NH + 2, JY = N + 2, SIZE = (N + 2) * JY * HX;
    __device__ static __forceinline__ int at(int k, int j, int h) { return ((k + 1) * JY + (j + 1)) * HX + (h + 1); }
};

template <int N>
struct Per {
    static constexpr int HALF = N * N * N / 2, PER = HALF / 256;  // cells of one colour per thread
};

template <typename T, int N>
__device__ __forceinline__ void face_ids(const LV<T> &L, int blk, int nbk[6]) {
    const int4 a = L.nbr[2 * blk], b = L.nbr[2 * blk + 1];
    nbk[0] = a.x;
    nbk[1] = a.y;
    nbk[2] = a.z;
    nbk[3] = a.w;
    nbk[4] = b.x;
    nbk[5] = b.y;
}

// The per-block table loads (rhs flag, leaf flag, position, face
// neighbours, record offset) are issued together and waited for once: the
// empty asm takes them all as operands before the early exits, which keeps
// the compiler from sinking the later ones below the exit tests (one
// dependent memory round trip instead of two or three per launch).
__device__ __forceinline__ void tables_loaded(int act, int leaf, int4 P, const int *nbk, int mo) {
    asm volatile("" ::"s"(act), "s"(leaf), "s"(P.x), "s"(P.y), "s"(P.z), "s"(nbk[0]), "s"(nbk[1]), "s"(nbk[2]),
                 "s"(nbk[3]), "s"(nbk[4]), "s"(nbk[5]), "s"(mo));
}

__device__ __forceinline__ bool any_coarser(const int *nbk) {
    return nbk[0] == -1 || nbk[1] == -1 || nbk[2] == -1 || nbk[3] == -1 || nbk[4] == -1 || nbk[5] == -1;
}

// Ghost values at the faces of a block that border a coarser level (-1).
// Each cell of colour `col` on such a face reads exactly one halo slot of
// the other-colour tile across that face; the slot receives the refinement
// boundary interpolation seen by that cell.  Runs after staging (it reads
// the inward neighbour from the tile); domain faces are filled while
// staging.  The NT calling threads take N*N/2 entries of a face each, so
// that the coarser faces of a block (up to NT/(N*N/2) at a time) are filled
// side by side, each a chain of two dependent loads (level table, value).
template <typename T, int N, int NT = 256>
__device__ void coarser_face_ghosts(T *tile, const LV<T> &Lc, const T *__restrict__ own_col, const T *phic,
                                    const int *nbk, int4 P, int col, int t) {
    using CT = ColTile<N>;
    constexpr int NH = N / 2, FE = N * NH, FPP = NT / FE > 0 ? NT / FE : 1;
    int mask = 0;
#pragma unroll
    for (int d = 0; d < 6; d++) mask |= (nbk[d] == -1 ? 1 : 0) << d;
    const int ncf = __popc(mask), slotf = t / FE, e = t % FE;
    if (slotf >= FPP) return;
#pragma unroll 1
    for (int f0 = 0; f0 < ncf; f0 += FPP) {
        const int fi = f0 + slotf;
        if (fi >= ncf) break;
        int m = mask;  // face d: the fi-th coarser face
        for (int r = 0; r < fi; r++) m &= m - 1;
        const int d = __ffs(m) - 1;
        const int ax = d >> 1, s = (d & 1) ? 1 : -1;
        int i, j, k, slot;
        if (ax == 0) {
            const int want = s < 0 ? 0 : 1;  // parity (col+j+k)&1 of rows whose cell touches the face
            k = e / NH;
            j = 2 * (e % NH) + ((col + k + want) & 1);
            i = s < 0 ? 0 : N - 1;
            slot = CT::at(k, j, s < 0 ? -1 : NH);
        } else if (ax == 1) {
            k = e / NH;
            const int h = e % NH;
            j = s < 0 ? 0 : N - 1;
            i = 2 * h + ((col + j + k) & 1);
            slot = CT::at(k, s < 0 ? -1 : N, h);
        } else {
            j = e / NH;
            const int h = e % NH;
            k = s < 0 ? 0 : N - 1;
            i = 2 * h + ((col + j + k) & 1);
            slot = CT::at(s < 0 ? -1 : N, j, h);
        }
        T ghost = T(0);
        if (phic) {
            const T own = own_col[(k * N + j) * NH + (i >> 1)];
            int c[3] = {i, j, k};
            c[ax] -= s;  // inward neighbour, other colour, inside the block
            const T f2 = tile[CT::at(c[2], c[1], c[0] >> 1)];
            ghost = cf_ghost<T, 3, N>(Lc, phic, P.x * N + i, P.y * N + j, P.z * N + k, ax, s, own, f2);
        }
        tile[slot] = ghost;
    }
}

// Halo value across face d of the block for the reading cell (i, j, k) of
// the other colour: the neighbour block's cell, or at a domain face the
// Dirichlet ghost 2 phi_b - own (own: the reading cell's value; 0 for
// ZERO) or the zero-flux ghost own; 0 at a coarser-level face (filled later
// by coarser_face_ghosts).  Split in two so that a thread's face loads all
// leave before any is waited for: halo_load issues both loads from valid
// addresses whatever the face type (a: neighbour cell or own value; b: face
// value, else a repeat of a's address), halo_pick selects the result.
template <typename T>
struct HaloLoads {
    T a, b;
};

template <typename T, int N, bool ZERO>
__device__ __forceinline__ HaloLoads<T> halo_load(const LV<T> &L, const T *__restrict__ phi,
                                                  const T *__restrict__ own_col, int nb, long long nidx, int d,
                                                  int4 P, int i, int j, int k, int oidx) {
    const bool zf = zero_flux(L.neumann, d >> 1, (d & 1) ? 1 : -1);
    const T *src = nb >= 0 ? phi + (long long)nb * Blk<3, N>::CPB + nidx : own_col + oidx;
    const T *bsrc = nb == -2 && !zf && L.bcv ? L.bcv + face_slot<3>(d >> 1, (d & 1) ? 1 : -1, P.x * N + i,
                                                                     P.y * N + j, P.z * N + k, L.n, L.nface)
                                             : src;
    return {ZERO ? T(0) : *src, *bsrc};
}

template <typename T, bool ZERO>
__device__ __forceinline__ T halo_pick(const LV<T> &L, HaloLoads<T> h, int nb, int d) {
    const bool zf = zero_flux(L.neumann, d >> 1, (d & 1) ? 1 : -1);
    const T bv = nb == -2 && !zf && L.bcv ? h.b : T(0);
    if (ZERO) return nb == -2 && !zf ? T(2) * bv : T(0);
    return nb >= 0 ? h.a : (nb == -1 ? T(0) : (zf ? h.a : T(2) * bv - h.a));
}

// colour slot m of thread t: the thread's cells are t + NT m, or with V2
// adjacent pairs 2 (t + NT (m / 2)) + m % 2
template <int NT, bool V2>
__device__ __forceinline__ int cell_of(int t, int m) {
    return V2 ? 2 * (t + NT * (m >> 1)) + (m & 1) : t + NT * m;
}

// the PER cells of thread t (slots of cell_of) from p, and back; with V2 one
// 2-element vector access per pair (p even-aligned); NTL: non-temporal loads
template <typename T, int PER, int NT, bool V2, bool NTL = false>
__device__ __forceinline__ void load_cells(const T *p, int t, T *out) {
    typedef T T2 __attribute__((ext_vector_type(2)));
    if (V2) {
#pragma unroll
        for (int m = 0; m < PER; m += 2) {
            const T2 *a = reinterpret_cast<const T2 *>(p + cell_of<NT, true>(t, m));
            const T2 w = NTL ? __builtin_nontemporal_load(a) : *a;
            out[m] = w.x;
            out[m + 1] = w.y;
        }
    } else {
#pragma unroll
        for (int m = 0; m < PER; m++) out[m] = NTL ? __builtin_nontemporal_load(p + t + NT * m) : p[t + NT * m];
    }
}

template <typename T, int PER, int NT, bool V2>
__device__ __forceinline__ void store_cells(T *p, int t, const T *v) {
    typedef T T2 __attribute__((ext_vector_type(2)));
    if (V2) {
#pragma unroll
        for (int m = 0; m < PER; m += 2) {
            T2 w;
            w.x = v[m];
            w.y = v[m + 1];
            *reinterpret_cast<T2 *>(p + cell_of<NT, true>(t, m)) = w;
        }
    } else {
#pragma unroll
        for (int m = 0; m < PER; m++) p[t + NT * m] = v[m];
    }
}

// paired cells are used on 16^3 blocks (an even number of cells per thread)
constexpr bool kCellPairs = true;
template <int N>
constexpr bool cell_pairs() {
    return kCellPairs && N == 16;
}

// Stage colour `col` of block `blk` and its face halos into a ColTile, the
// halos at domain faces as the Dirichlet ghosts seen by the cells of the
// other colour.  All global loads of the thread are issued before the LDS
// writes.
// NT threads stage the colour (t < NT); the faces take the first N*N.
// With V2 a thread's cells come in adjacent pairs (slots of cell_of), the
// staged interior loaded with one 2-element vector access per pair.
// own: the reading colour's values for the domain ghosts (colour-compact,
// (k N + j) N/2 + i/2; default: that colour of the block in phi).
template <typename T, int N, bool ZERO, int NT = 256, bool V2 = false>
__device__ __forceinline__ void stage_colour(T *tile, const LV<T> &L, const T *__restrict__ phi, int blk,
                                             const int *nbk, int4 P, int col, int t,
                                             const T *interior = nullptr, const T *own = nullptr) {
    using B = Blk<3, N>;
    using CT = ColTile<N>;
    constexpr int NH = N / 2, PER = B::HALF / NT;
    const int oc = col * B::HALF, uc = (1 - col) * B::HALF;
    const T *__restrict__ own_col = own ? own : phi + (long long)blk * B::CPB + uc;
    T r[PER];
    if (ZERO) {
        for (int e = t; e < CT::SIZE; e += NT) tile[e] = T(0);
    } else if (interior) {
#pragma unroll
        for (int m = 0; m < PER; m++) r[m] = interior[m];
    } else {
        load_cells<T, PER, NT, V2>(phi + (long long)blk * B::CPB + oc, t, r);
    }
    const int ucol = 1 - col;
    const int fh = t % NH, fr = t / NH;  // y/z face entry (N*NH <= 256)
    const int xj = t % N, xk = t / N;    // x face entry (N*N <= 256)
    const bool fz = t < N * NH, fx = t < N * N;
    HaloLoads<T> hy0{}, hy1{}, hz0{}, hz1{}, hx{};
    if (fz) {
        // y faces: entry (k = fr, h = fh); z faces: entry (j = fr, h = fh)
        const int ky = fr, jz = fr;
        hy0 = halo_load<T, N, ZERO>(L, phi, own_col, nbk[2], oc + (ky * N + N - 1) * NH + fh, 2, P,
                                    2 * fh + ((ucol + ky) & 1), 0, ky, (ky * N) * NH + fh);
        hy1 = halo_load<T, N, ZERO>(L, phi, own_col, nbk[3], oc + (ky * N) * NH + fh, 3, P,
                                    2 * fh + ((ucol + N - 1 + ky) & 1), N - 1, ky, (ky * N + N - 1) * NH + fh);
        hz0 = halo_load<T, N, ZERO>(L, phi, own_col, nbk[4], oc + ((N - 1) * N + jz) * NH + fh, 4, P,
                                    2 * fh + ((ucol + jz) & 1), jz, 0, jz * NH + fh);
        hz1 = halo_load<T, N, ZERO>(L, phi, own_col, nbk[5], oc + jz * NH + fh, 5, P,
                                    2 * fh + ((ucol + jz + N - 1) & 1), jz, N - 1, ((N - 1) * N + jz) * NH + fh);
    }
    // x faces: entry (j = xj, k = xk).  A row's reading cells sit at
    // i = 0 or at i = N-1, by its parity: it reads exactly one of its two x
    // halos (x- when xp = 0, else x+), the only one loaded
    const int xp = (ucol + xj + xk) & 1, nbx = xp ? nbk[1] : nbk[0];
    if (fx) {
        hx = halo_load<T, N, ZERO>(L, phi, own_col, nbx, oc + (xk * N + xj) * NH + (xp ? 0 : NH - 1), xp, P,
                                   xp ? N - 1 : 0, xj, xk, (xk * N + xj) * NH + (xp ? NH - 1 : 0));
    }
    // one wait for all face loads (the empty asm consumes them; without it
    // the compiler moves each face's second load into a branch and waits
    // for it there, one round trip per face)
    asm volatile("" ::"v"(hy0.a), "v"(hy0.b), "v"(hy1.a), "v"(hy1.b), "v"(hz0.a), "v"(hz0.b), "v"(hz1.a),
                 "v"(hz1.b), "v"(hx.a), "v"(hx.b));
    const T y0 = halo_pick<T, ZERO>(L, hy0, nbk[2], 2), y1 = halo_pick<T, ZERO>(L, hy1, nbk[3], 3);
    const T z0 = halo_pick<T, ZERO>(L, hz0, nbk[4], 4), z1 = halo_pick<T, ZERO>(L, hz1, nbk[5], 5);
    const T xv = halo_pick<T, ZERO>(L, hx, nbx, xp);
    if (!ZERO) {
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int q = cell_of<NT, V2>(t, m);
            tile[CT::at(q / (NH * N), (q / NH) % N, q % NH)] = r[m];
        }
    } else {
        __syncthreads();  // the zero fill before the halo writes
    }
    if (fz) {
        tile[CT::at(fr, -1, fh)] = y0;
        tile[CT::at(fr, N, fh)] = y1;
        tile[CT::at(-1, fr, fh)] = z0;
        tile[CT::at(N, fr, fh)] = z1;
    }
    if (fx) tile[CT::at(xk, xj, xp ? NH : -1)] = xv;
}

// the 6 neighbour values of cell q of colour `col` from the other-colour tile
template <typename T, int N>
__device__ __forceinline__ void tile_neighbours(const T *tile, int col, int q, int &i, int &j, int &k, T v[6]) {
    using CT = ColTile<N>;
    constexpr int NH = N / 2;
    const int h = q % NH;
    j = (q / NH) % N;
    k = q / (NH * N);
    const int par = (col + j + k) & 1;
    i = 2 * h + par;
    v[0] = tile[CT::at(k, j, h - 1 + par)];
    v[1] = tile[CT::at(k, j, h + par)];
    v[2] = tile[CT::at(k, j - 1, h)];
    v[3] = tile[CT::at(k, j + 1, h)];
    v[4] = tile[CT::at(k - 1, j, h)];
    v[5] = tile[CT::at(k + 1, j, h)];
}

// red-black half sweep, NT threads per block (V2: cells in adjacent pairs).
// U (FP32 sweeps only): the FP64 level of a mixed-precision solve; the
// block's FP64 values take the update phi += e from the swept colour's new
// values and the other colour's staged ones (k_gs_half3_update).  keep: the
// swept colour is stored as well and only leaf blocks are updated (levels
// of adaptive trees, whose values finer levels still read as ghosts)
template <typename T, int N, int NT = 256, bool V2 = false>
__device__ __forceinline__ void gs_half3_body(const LV<T> &L, const LV<T> &Lc, int color, int blk, int rhs, T *tile,
                                              const LV<double> *U = nullptr, int keep = 0) {
    using B = Blk<3, N>;
    constexpr int PER = B::HALF / NT;
    const int4 P = L.pos[blk];
    int nbk[6];
    face_ids<T, N>(L, blk, nbk);
    const int mo = L.map_off ? L.map_off[blk] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    const int leaf = U && keep ? L.leaf[blk] : 1;
    tables_loaded(act, leaf, P, nbk, mo);
    if (!act) return;
    T *__restrict__ phi = L.phi + (long long)rhs * L.fstride;
    const long long base = (long long)blk * B::CPB;
    const T *__restrict__ gm = L.g + (long long)rhs * L.fstride + base + color * B::HALF;
    T gv[PER];
    int ri[PER];
    // g is read once per sweep: in FP64, non-temporal loads keep it from
    // evicting the phi lines that neighbouring blocks read as halos (41.6
    // against 44.7 us at 256^3); the FP32 sweep is faster with plain loads
    // (26.5 against 27.2 us)
    load_cells<T, PER, NT, V2, sizeof(T) == 8>(gm, threadIdx.x, gv);
#pragma unroll
    for (int m = 0; m < PER; m++) ri[m] = mo >= 0 ? L.map[mo + color * B::HALF + cell_of<NT, V2>(threadIdx.x, m)] : -1;
    // the cells' own values for their ghosts: phi, or after a fused
    // prolongation and red half sweep (black) the prolonged values in L.own
    const T *own = L.own ? L.own + (long long)rhs * L.fstride + base + color * B::HALF : nullptr;
    stage_colour<T, N, false, NT, V2>(tile, L, phi, blk, nbk, P, 1 - color, threadIdx.x, nullptr, own);
    __syncthreads();
    T *__restrict__ dst = phi + base + color * B::HALF;
    if (any_coarser(nbk)) {
        const T *phic = Lc.phi ? Lc.phi + (long long)rhs * Lc.fstride : nullptr;
        coarser_face_ghosts<T, N, NT>(tile, Lc, own ? own : dst, phic, nbk, P, color, threadIdx.x);
        __syncthreads();
    }
    const T inv6 = T(1) / T(6);
    T nv[PER];
#pragma unroll
    for (int m = 0; m < PER; m++) {
        const int q = cell_of<NT, V2>(threadIdx.x, m);
        int i, j, k;
        T v[6];
        tile_neighbours<T, N>(tile, color, q, i, j, k, v);
        if (ri[m] < 0) {
            nv[m] = (((v[0] + v[1]) + (v[2] + v[3])) + (v[4] + v[5]) - L.dx2 * gv[m]) * inv6;
        } else {
            const T *r = L.rec + 8 * (long long)ri[m];
            T s = T(0);
#pragma unroll
            for (int d = 0; d < 6; d++) s += r[d] * v[d];
            const T bt = L.b ? L.b[ri[m]] : T(0);
            nv[m] = (gv[m] - bt - s) * r[7];
        }
    }
    if (!U || keep) store_cells<T, PER, NT, V2>(dst, threadIdx.x, nv);
    if (!U || !leaf) return;
    // phi += e on both colours, in FP64 (k_update's arithmetic); without
    // keep the swept colour's e is not stored
    constexpr int NH = N / 2;
    using CT = ColTile<N>;
    double *p64 = U->phi + (long long)rhs * U->fstride + base;
    double sw[PER], ot[PER];
    load_cells<double, PER, NT, V2, true>(p64 + color * B::HALF, threadIdx.x, sw);
    load_cells<double, PER, NT, V2, true>(p64 + (1 - color) * B::HALF, threadIdx.x, ot);
#pragma unroll
    for (int m = 0; m < PER; m++) {
        const int q = cell_of<NT, V2>(threadIdx.x, m);
        sw[m] += (double)nv[m];
        ot[m] += (double)tile[CT::at(q / (NH * N), (q / NH) % N, q % NH)];
    }
    store_cells<double, PER, NT, V2>(p64 + color * B::HALF, threadIdx.x, sw);
    store_cells<double, PER, NT, V2>(p64 + (1 - color) * B::HALF, threadIdx.x, ot);
}

template <typename T, int N, int NT, bool V2>
__global__ __launch_bounds__(NT) void k_gs_half3(LV<T> L, LV<T> Lc, int color) {
    __shared__ T tile[ColTile<N>::SIZE];
    gs_half3_body<T, N, NT, V2>(L, Lc, color, block_of(L), rhs_of(L), tile);
}

// The last half sweep (black) of a level in the FP32 correction's final
// V-cycle, fused with the FP64 update phi += e of the level's leaf blocks
// that follows the cycle (k_update): the black cells add their new values,
// the red cells the values staged for the sweep, which it does not change.
// keep = 0 (the finest level: every block a leaf, no finer level): the
// black correction values themselves are not stored, since the next defect
// overwrites the correction on every leaf cell before anything reads it;
// keep = 1 (coarser levels of adaptive trees): they are stored, parent
// blocks and finer levels' ghosts read them.  Same FP64 bits as the half
// sweep followed by k_update.
template <int N, int NT, bool V2>
__global__ __launch_bounds__(NT) void k_gs_half3_update(LV<float> L, LV<float> Lc, LV<double> U, int keep) {
    __shared__ float tile[ColTile<N>::SIZE];
    gs_half3_body<float, N, NT, V2>(L, Lc, 1, block_of(L), rhs_of(L), tile, &U, keep);
}

// L phi at the PER cells of colour `col` owned by this thread, from the
// other-colour tile (already staged, ghosts filled); `own` their values.
template <typename T, int N, int NT = 256, bool V2 = false>
__device__ __forceinline__ void tile_op(const LV<T> &L, const T *tile, const int *ri, int col, const T *own, T *out,
                                        int t) {
    constexpr int PER = Blk<3, N>::HALF / NT;
#pragma unroll
    for (int m = 0; m < PER; m++) {
        const int q = cell_of<NT, V2>(t, m);
        int i, j, k;
        T v[6];
        tile_neighbours<T, N>(tile, col, q, i, j, k, v);
        if (ri[m] < 0) {
            out[m] = L.inv_dx2 * ((((v[0] + v[1]) + (v[2] + v[3])) + (v[4] + v[5])) - T(6) * own[m]);
        } else {
            const T *r = L.rec + 8 * (long long)ri[m];
            T s = T(0);
#pragma unroll
            for (int d = 0; d < 6; d++) s += r[d] * v[d];
            out[m] = s + r[6] * own[m] + (L.b ? L.b[ri[m]] : T(0));
        }
    }
}

// Pass over colour `col` of block `blk`: stage the other colour (from HBM,
// or from `interior` registers), fill open-face ghosts, apply L.  The tile
// stays live until the caller's next __syncthreads().
template <typename T, int N, bool ZERO>
__device__ __forceinline__ void colour_pass(const LV<T> &L, const LV<T> &Lc, const T *phi, const T *phic, T *tile,
                                            int blk, const int *nbk, int4 P, const int *ri, int col, const T *own,
                                            const T *interior, T *out) {
    stage_colour<T, N, ZERO>(tile, L, phi, blk, nbk, P, 1 - col, threadIdx.x, interior);
    __syncthreads();
    if (!ZERO && any_coarser(nbk)) {
        coarser_face_ghosts<T, N>(tile, Lc, phi + (long long)blk * Blk<3, N>::CPB + col * Blk<3, N>::HALF, phic, nbk,
                                  P, col, threadIdx.x);
        __syncthreads();
    }
    tile_op<T, N>(L, tile, ri, col, own, out, threadIdx.x);
}

// own values of colour 1 read back from the colour-1 tile of the first pass
template <typename T, int N>
__device__ __forceinline__ void own_from_tile(const T *tile, T *own) {
    constexpr int NH = N / 2, PER = Per<N>::PER;
#pragma unroll
    for (int m = 0; m < PER; m++) {
        const int q = threadIdx.x + 256 * m;
        own[m] = tile[ColTile<N>::at(q / (NH * N), (q / NH) % N, q % NH)];
    }
}

template <int N>
__device__ __forceinline__ void q_to_ijk(int col, int q, int &i, int &j, int &k) {
    constexpr int NH = N / 2;
    const int h = q % NH;
    j = (q / NH) % N;
    k = q / (NH * N);
    i = 2 * h + ((col + j + k) & 1);
}

// The kernels below read each colour array of the block once from HBM:
// pass 0 stages colour 1 (which pass 1 then takes its own values from) and
// pass 1 stages colour 0 from the registers that held its own values.

// FAS restriction, 3D: residual of every cell, then the 2x2x2 means of phi
// and r through a natural-order LDS array.  phi_c goes to Lc.old, and to
// Lc.phi as well unless `into_old`.
template <typename T, int N, int NC>
__device__ __forceinline__ void restrict_fas3_body(const LV<T> &L, const LV<T> &Lc, int into_old, int blk, int rhs, T *sm) {
    using B = Blk<3, N>;
    constexpr int PER = Per<N>::PER, H = N / 2, NCELL = H * H * H, CPER = (NCELL + 255) / 256;
    const int4 P = L.pos[blk];
    int nbk[6];
    face_ids<T, N>(L, blk, nbk);
    const int mo = L.map_off ? L.map_off[blk] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    tables_loaded(act, 1, P, nbk, mo);
    if (!act) return;
    const T *__restrict__ phi = L.phi + (long long)rhs * L.fstride;
    const T *__restrict__ g = L.g + (long long)rhs * L.fstride;
    const T *phic = Lc.phi + (long long)rhs * Lc.fstride;
    const long long base = (long long)blk * B::CPB;
    T own0[PER], own1[PER], r0[PER], r1[PER], gv[PER];
    int ri[PER];
    // colour 0
#pragma unroll
    for (int m = 0; m < PER; m++) {
        const int s = threadIdx.x + 256 * m;
        own0[m] = phi[base + s];
        gv[m] = g[base + s];
        ri[m] = mo >= 0 ? L.map[mo + s] : -1;
    }
    colour_pass<T, N, false>(L, Lc, phi, phic, sm, blk, nbk, P, ri, 0, own0, nullptr, r0);
    own_from_tile<T, N>(sm, own1);
#pragma unroll
    for (int m = 0; m < PER; m++) r0[m] = gv[m] - r0[m];
    __syncthreads();
    // colour 1
#pragma unroll
    for (int m = 0; m < PER; m++) {
        const int s = B::HALF + threadIdx.x + 256 * m;
        gv[m] = g[base + s];
        ri[m] = mo >= 0 ? L.map[mo + s] : -1;
    }
    colour_pass<T, N, false>(L, Lc, phi, phic, sm, blk, nbk, P, ri, 1, own1, own0, r1);
#pragma unroll
    for (int m = 0; m < PER; m++) r1[m] = gv[m] - r1[m];
    __syncthreads();
    // 2x2x2 means of r, then of phi, through natural-order LDS
    T rc[CPER], pc[CPER];
#pragma unroll
    for (int pass = 0; pass < 2; pass++) {
#pragma unroll
        for (int m = 0; m < PER; m++) {
            int i, j, k;
            q_to_ijk<N>(0, threadIdx.x + 256 * m, i, j, k);
            sm[(k * N + j) * N + i] = pass == 0 ? r0[m] : own0[m];
            q_to_ijk<N>(1, threadIdx.x + 256 * m, i, j, k);
            sm[(k * N + j) * N + i] = pass == 0 ? r1[m] : own1[m];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < CPER; m++) {
            const int cc = threadIdx.x + 256 * m;
            T s = T(0);
            if (cc < NCELL) {
                const int ci = cc % H, cj = (cc / H) % H, ck = cc / (H * H);
#pragma unroll
                for (int ch = 0; ch < 8; ch++)
                    s += sm[((2 * ck + ((ch >> 2) & 1)) * N + 2 * cj + ((ch >> 1) & 1)) * N + 2 * ci + (ch & 1)];
            }
            if (pass == 0) rc[m] = s;
            else pc[m] = s;
        }
        __syncthreads();
    }
    T *oldw = Lc.old + (long long)rhs * Lc.fstride, *phiw = Lc.phi + (long long)rhs * Lc.fstride;
    T *gw = Lc.g + (long long)rhs * Lc.fstride;
    const int C0[3] = {P.x * H, P.y * H, P.z * H};
    const int pb = block_at<T, 3>(Lc, C0[0] / NC, C0[1] / NC, C0[2] / NC);
    if (pb < 0) return;  // excluded by construction: every block has a parent
    const T inv = T(0.125);
#pragma unroll
    for (int m = 0; m < CPER; m++) {
        const int cc = threadIdx.x + 256 * m;
        if (cc >= NCELL) continue;
        const int ci = cc % H, cj = (cc / H) % H, ck = cc / (H * H);
        const int gi = C0[0] + ci, gj = C0[1] + cj, gk = C0[2] + ck;
        const long long o = (long long)pb * Blk<3, NC>::CPB + split_of<3, NC>(gi % NC, gj % NC, gk % NC);
        const T pv = pc[m] * inv;
        oldw[o] = pv;
        if (!into_old) phiw[o] = pv;
        gw[o] = rc[m] * inv;
    }
}

template <typename T, int N, int NC>
__global__ __launch_bounds__(256) void k_restrict_fas3(LV<T> L, LV<T> Lc, int into_old) {
    using B = Blk<3, N>;
    constexpr int SM = ColTile<N>::SIZE > B::CPB ? ColTile<N>::SIZE : B::CPB;
    __shared__ T sm[SM];
    restrict_fas3_body<T, N, NC>(L, Lc, into_old, block_of(L), rhs_of(L), sm);
}

// FAS rhs on parent blocks (g = L phi + g) and old = phi, 3D
template <typename T, int N>
__device__ __forceinline__ void fas_rhs3_body(const LV<T> &L, const LV<T> &Lc, int do_rhs, int blk, int rhs, T *tile) {
    using B = Blk<3, N>;
    constexpr int PER = Per<N>::PER;
    const int leaf = L.leaf[blk];
    const int4 P = L.pos[blk];
    int nbk[6];
    face_ids<T, N>(L, blk, nbk);
    const int mo = L.map_off ? L.map_off[blk] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    tables_loaded(act, leaf, P, nbk, mo);
    if (!act) return;
    T *phi = L.phi + (long long)rhs * L.fstride;
    T *g = L.g + (long long)rhs * L.fstride;
    T *old = L.old + (long long)rhs * L.fstride;
    const long long base = (long long)blk * B::CPB;
    if (leaf || !do_rhs) {
        for (int s = threadIdx.x; s < B::CPB; s += 256) old[base + s] = phi[base + s];
        return;
    }
    const T *phic = Lc.phi ? Lc.phi + (long long)rhs * Lc.fstride : nullptr;
    T own0[PER], own1[PER], lp[PER], gv[PER];
    int ri[PER];
#pragma unroll
    for (int c = 0; c < 2; c++) {
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int s = c * B::HALF + threadIdx.x + 256 * m;
            if (c == 0) own0[m] = phi[base + s];
            gv[m] = g[base + s];
            ri[m] = mo >= 0 ? L.map[mo + s] : -1;
        }
        colour_pass<T, N, false>(L, Lc, phi, phic, tile, blk, nbk, P, ri, c, c == 0 ? own0 : own1,
                                 c == 0 ? nullptr : own0, lp);
        if (c == 0) own_from_tile<T, N>(tile, own1);
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int s = c * B::HALF + threadIdx.x + 256 * m;
            g[base + s] = lp[m] + gv[m];
            old[base + s] = c == 0 ? own0[m] : own1[m];
        }
        __syncthreads();
    }
}

template <typename T, int N>
__global__ __launch_bounds__(256) void k_fas_rhs3(LV<T> L, LV<T> Lc, int do_rhs) {
    __shared__ T tile[ColTile<N>::SIZE];
    fas_rhs3_body<T, N>(L, Lc, do_rhs, block_of(L), rhs_of(L), tile);
}

// ------------------------------------------- colour-pair variants (3D)
// Workgroups of 2 NTC threads in which wave group c = threadIdx.x / NTC owns
// the cells of colour c (NTC = 256; 512 in the FAS right-hand side of small
// launches on 16^3 blocks).  Each group stages its own colour, with the
// halos seen by the other colour, into its own tile, so both tiles fill in
// one round of loads; after the refinement-boundary ghosts each group
// applies L to its colour from the other group's tile.  The arithmetic is
// that of the two-pass kernels above, term by term, so the results are the
// same bits; only the latency differs (one dependent load round instead of
// two).
template <typename T, int N>
struct PairTiles {
    static constexpr int SIZE = 2 * ColTile<N>::SIZE;
};

// L phi at this thread's HALF/NTC cells of colour c; `own` holds their
// values (registers), `tiles` two ColTiles.  Every thread of the workgroup
// calls it.  RELOAD: own is read back from the thread's staged tile after
// the barrier (the same values), so its registers are free while the halos
// are in flight.
template <typename T, int N, int NTC, bool RELOAD = false>
__device__ __forceinline__ void pair_op(const LV<T> &L, const LV<T> &Lc, const T *phi, const T *phic, T *tiles,
                                        int blk, const int *nbk, int4 P, const int *ri, T *own, T *out) {
    constexpr bool V2 = cell_pairs<N>();
    constexpr int PER = Blk<3, N>::HALF / NTC, NH = N / 2;
    const int c = threadIdx.x / NTC, t = threadIdx.x % NTC;
    T *mine = tiles + c * ColTile<N>::SIZE, *other = tiles + (1 - c) * ColTile<N>::SIZE;
    stage_colour<T, N, false, NTC, V2>(mine, L, phi, blk, nbk, P, c, t, own);
    __syncthreads();
    if (any_coarser(nbk)) {
        coarser_face_ghosts<T, N, NTC>(other, Lc, phi + (long long)blk * Blk<3, N>::CPB + c * Blk<3, N>::HALF, phic,
                                       nbk, P, c, t);
        __syncthreads();
    }
    if (RELOAD) {
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int q = cell_of<NTC, V2>(t, m);
            own[m] = mine[ColTile<N>::at(q / (NH * N), (q / NH) % N, q % NH)];
        }
    }
    tile_op<T, N, NTC, V2>(L, other, ri, c, own, out, t);
}

// LATE: g is loaded after the stencil, so its registers are not live across
// the staging and three workgroups fit a CU (LDS and registers); pays where
// a launch has many workgroups per CU, costs one dependent load where it
// has few
template <typename T, int N, int NC, int NTC, bool LATE>
__global__ __launch_bounds__(2 * NTC) __attribute__((amdgpu_waves_per_eu(LATE ? 6 : 1))) void k_restrict_fas3_pair(
    LV<T> L, LV<T> Lc, int into_old) {
    using B = Blk<3, N>;
    constexpr int PER = B::HALF / NTC, H = N / 2, NCELL = H * H * H;
    static_assert(NCELL <= 2 * NTC, "one coarse cell per thread");
    constexpr bool V2 = cell_pairs<N>();
    constexpr int NF = LATE ? 1 : 2;  // natural-order arrays held at once
    constexpr int SM = PairTiles<T, N>::SIZE > NF * B::CPB ? PairTiles<T, N>::SIZE : NF * B::CPB;
    __shared__ T sm[SM];
    const int blk = block_of(L), rhs = rhs_of(L);
    const int c = threadIdx.x / NTC, t = threadIdx.x % NTC;
    const int4 P = L.pos[blk];
    int nbk[6];
    face_ids<T, N>(L, blk, nbk);
    const int mo = L.map_off ? L.map_off[blk] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    tables_loaded(act, 1, P, nbk, mo);
    if (!act) return;
    const T *__restrict__ phi = L.phi + (long long)rhs * L.fstride;
    const T *__restrict__ g = L.g + (long long)rhs * L.fstride;
    const T *phic = Lc.phi + (long long)rhs * Lc.fstride;
    const long long base = (long long)blk * B::CPB + c * B::HALF;
    T own[PER], r[PER], gv[PER];
    int ri[PER];
    load_cells<T, PER, NTC, V2>(phi + base, t, own);
    if (!LATE) load_cells<T, PER, NTC, V2>(g + base, t, gv);
#pragma unroll
    for (int m = 0; m < PER; m++) ri[m] = mo >= 0 ? L.map[mo + c * B::HALF + cell_of<NTC, V2>(t, m)] : -1;
    pair_op<T, N, NTC, LATE>(L, Lc, phi, phic, sm, blk, nbk, P, ri, own, r);
    if (LATE) load_cells<T, PER, NTC, V2>(g + base, t, gv);
#pragma unroll
    for (int m = 0; m < PER; m++) r[m] = gv[m] - r[m];
    // the tiles become natural-order arrays of r and phi: both at once, or
    // with LATE one after the other (one 32 KB array: three workgroups per
    // CU fit the LDS)
    const int cc = threadIdx.x, ci = cc % H, cj = (cc / H) % H, ck = cc / (H * H);
    T sums[2];
#pragma unroll
    for (int f0 = 0; f0 < 2; f0 += NF) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < PER; m++) {
            int i, j, k;
            q_to_ijk<N>(c, cell_of<NTC, V2>(t, m), i, j, k);
#pragma unroll
            for (int f = f0; f < f0 + NF; f++) sm[(f - f0) * B::CPB + (k * N + j) * N + i] = f == 0 ? r[m] : own[m];
        }
        __syncthreads();
#pragma unroll
        for (int f = f0; f < f0 + NF; f++) {
            T s = T(0);
            if (cc < NCELL) {
#pragma unroll
                for (int ch = 0; ch < 8; ch++)
                    s += sm[(f - f0) * B::CPB +
                            ((2 * ck + ((ch >> 2) & 1)) * N + 2 * cj + ((ch >> 1) & 1)) * N + 2 * ci + (ch & 1)];
            }
            sums[f] = s;
        }
    }
    if (cc >= NCELL) return;
    T *oldw = Lc.old + (long long)rhs * Lc.fstride, *phiw = Lc.phi + (long long)rhs * Lc.fstride;
    T *gw = Lc.g + (long long)rhs * Lc.fstride;
    const int C0[3] = {P.x * H, P.y * H, P.z * H};
    const int pb = block_at<T, 3>(Lc, C0[0] / NC, C0[1] / NC, C0[2] / NC);
    if (pb < 0) return;  // excluded by construction: every block has a parent
    const T inv = T(0.125);
    const int gi = C0[0] + ci, gj = C0[1] + cj, gk = C0[2] + ck;
    const long long o = (long long)pb * Blk<3, NC>::CPB + split_of<3, NC>(gi % NC, gj % NC, gk % NC);
    const T pv = sums[1] * inv;
    oldw[o] = pv;
    if (!into_old) phiw[o] = pv;
    gw[o] = sums[0] * inv;
}

template <typename T, int N, int NTC>
__global__ __launch_bounds__(2 * NTC) void k_fas_rhs3_pair(LV<T> L, LV<T> Lc, int do_rhs) {
    using B = Blk<3, N>;
    constexpr int PER = B::HALF / NTC;
    constexpr bool V2 = cell_pairs<N>();
    __shared__ T tiles[PairTiles<T, N>::SIZE];
    const int blk = block_of(L), rhs = rhs_of(L);
    const int c = threadIdx.x / NTC, t = threadIdx.x % NTC;
    const int leaf = L.leaf[blk];
    const int4 P = L.pos[blk];
    int nbk[6];
    face_ids<T, N>(L, blk, nbk);
    const int mo = L.map_off ? L.map_off[blk] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    tables_loaded(act, leaf, P, nbk, mo);
    if (!act) return;
    const T *phi = L.phi + (long long)rhs * L.fstride;
    T *g = L.g + (long long)rhs * L.fstride;
    T *old = L.old + (long long)rhs * L.fstride;
    if (leaf || !do_rhs) {
        const long long b0 = (long long)blk * B::CPB;
        for (int s = threadIdx.x; s < B::CPB; s += 2 * NTC) old[b0 + s] = phi[b0 + s];
        return;
    }
    const T *phic = Lc.phi ? Lc.phi + (long long)rhs * Lc.fstride : nullptr;
    const long long base = (long long)blk * B::CPB + c * B::HALF;
    T own[PER], lp[PER], gv[PER];
    int ri[PER];
    load_cells<T, PER, NTC, V2>(phi + base, t, own);
    load_cells<T, PER, NTC, V2>(g + base, t, gv);
#pragma unroll
    for (int m = 0; m < PER; m++) ri[m] = mo >= 0 ? L.map[mo + c * B::HALF + cell_of<NTC, V2>(t, m)] : -1;
    pair_op<T, N, NTC>(L, Lc, phi, phic, tiles, blk, nbk, P, ri, own, lp);
#pragma unroll
    for (int m = 0; m < PER; m++) lp[m] = lp[m] + gv[m];
    store_cells<T, PER, NTC, V2>(g + base, t, lp);
    store_cells<T, PER, NTC, V2>(old + base, t, own);
}

// FAS right-hand side fused with the first red half sweep of a coarse
// level (3D).  Entry state: phi = old on every block of the level (the
// restriction wrote both; on leaf blocks of adaptive trees old was copied
// from phi).  Both colour tiles are staged from old, which no workgroup
// writes here, so the red half sweep may overwrite phi meanwhile.  Each
// wave group applies L to its colour; on parent blocks g <- L phi + g (the
// FAS right-hand side, Sec. 2.2); then group 0 updates the red cells from
// the black tile with that g.  Term by term the arithmetic of k_fas_rhs3
// followed by k_gs_half3 on colour 0: the same bits.
template <typename T, int N, int NTC>
__global__ __launch_bounds__(2 * NTC) void k_fas_gs3_pair(LV<T> L, LV<T> Lc, int own_to_phi) {
    using B = Blk<3, N>;
    constexpr int PER = B::HALF / NTC;
    constexpr bool V2 = cell_pairs<N>();
    __shared__ T tiles[PairTiles<T, N>::SIZE];
    const int blk = block_of(L), rhs = rhs_of(L);
    const int c = threadIdx.x / NTC, t = threadIdx.x % NTC;
    const int leaf = L.leaf[blk];
    const int4 P = L.pos[blk];
    int nbk[6];
    face_ids<T, N>(L, blk, nbk);
    const int mo = L.map_off ? L.map_off[blk] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    tables_loaded(act, leaf, P, nbk, mo);
    if (!act) return;
    const T *old = L.old + (long long)rhs * L.fstride;
    T *phi = L.phi + (long long)rhs * L.fstride;
    T *g = L.g + (long long)rhs * L.fstride;
    const T *phic = Lc.phi ? Lc.phi + (long long)rhs * Lc.fstride : nullptr;
    const long long base = (long long)blk * B::CPB + c * B::HALF;
    T own[PER], lp[PER], gv[PER];
    int ri[PER];
    load_cells<T, PER, NTC, V2>(old + base, t, own);
    load_cells<T, PER, NTC, V2>(g + base, t, gv);
#pragma unroll
    for (int m = 0; m < PER; m++) ri[m] = mo >= 0 ? L.map[mo + c * B::HALF + cell_of<NTC, V2>(t, m)] : -1;
    pair_op<T, N, NTC>(L, Lc, old, phic, tiles, blk, nbk, P, ri, own, lp);
    if (!leaf) {
#pragma unroll
        for (int m = 0; m < PER; m++) gv[m] = lp[m] + gv[m];
        store_cells<T, PER, NTC, V2>(g + base, t, gv);
    }
    if (c != 0) {
        // black cells of a parent block: phi <- old, when the restriction
        // wrote old only (no workgroup reads phi of this level here)
        if (own_to_phi && !leaf) store_cells<T, PER, NTC, V2>(phi + base, t, own);
        return;
    }
    // red half sweep from the black tile (its ghosts were filled for the red cells)
    const T *tile = tiles + ColTile<N>::SIZE;
    const T inv6 = T(1) / T(6);
    T nv[PER];
#pragma unroll
    for (int m = 0; m < PER; m++) {
        const int q = cell_of<NTC, V2>(t, m);
        int i, j, k;
        T v[6];
        tile_neighbours<T, N>(tile, 0, q, i, j, k, v);
        if (ri[m] < 0) {
            nv[m] = (((v[0] + v[1]) + (v[2] + v[3])) + (v[4] + v[5]) - L.dx2 * gv[m]) * inv6;
        } else {
            const T *r = L.rec + 8 * (long long)ri[m];
            T sm = T(0);
#pragma unroll
            for (int d = 0; d < 6; d++) sm += r[d] * v[d];
            const T bt = L.b ? L.b[ri[m]] : T(0);
            nv[m] = (gv[m] - bt - sm) * r[7];
        }
    }
    store_cells<T, PER, NTC, V2>(phi + base, t, nv);
}

// ------------------------------------------- single-block level (3D)
// A level made of one 16^3 block (the level above an 8^3 coarsest grid)
// covers the domain: all six faces are domain faces, so its half sweeps need
// no other workgroup's values.  One workgroup of 1024 threads keeps both
// colours in LDS (a ColTile each, whose halos hold the ghosts seen by the
// other colour) and runs the level's steps of a V-cycle behind workgroup
// barriers instead of one launch each: on the way down the FAS right-hand
// side from `old`, `steps` red-black sweeps, then the residual and the
// restriction to the coarse grid; on the way up the sweeps alone.  Thread t
// owns the cell pair 2t, 2t+1 of each colour; its g values, record rows and
// boundary terms stay in registers.  The arithmetic is that of
// k_fas_gs3_pair, k_gs_half3 and k_restrict_fas3_pair term by term (the same
// bits).

// ghosts in `dst` (a colour's tile) for the cells of colour u at the domain
// faces, from their current values in `src` (colour u's tile): a zero-flux
// face copies the cell, a Dirichlet face reflects it about the face value
// (2 bv - value; bv = 0 without face data).  bv: [5][256] face values of the
// reading colour (y-, y+, z-, z+, x entries)
template <typename T>
__device__ __forceinline__ void sb_ghosts(T *dst, const T *src, const T *bv, int u, int nm, int t) {
    constexpr int N = 16, NH = 8;
    using CT = ColTile<N>;
    if (t < N * NH) {
        const int fh = t % NH, fr = t / NH;
        T a = src[CT::at(fr, 0, fh)];
        dst[CT::at(fr, -1, fh)] = zero_flux(nm, 1, -1) ? a : T(2) * bv[t] - a;
        a = src[CT::at(fr, N - 1, fh)];
        dst[CT::at(fr, N, fh)] = zero_flux(nm, 1, 1) ? a : T(2) * bv[256 + t] - a;
        a = src[CT::at(0, fr, fh)];
        dst[CT::at(-1, fr, fh)] = zero_flux(nm, 2, -1) ? a : T(2) * bv[512 + t] - a;
        a = src[CT::at(N - 1, fr, fh)];
        dst[CT::at(N, fr, fh)] = zero_flux(nm, 2, 1) ? a : T(2) * bv[768 + t] - a;
    }
    if (t < N * N) {
        const int xj = t % N, xk = t / N, xp = (u + xj + xk) & 1;
        const T a = src[CT::at(xk, xj, xp ? NH - 1 : 0)];
        dst[CT::at(xk, xj, xp ? NH : -1)] = zero_flux(nm, 0, xp ? 1 : -1) ? a : T(2) * bv[1024 + t] - a;
    }
}

template <typename T, bool FAS, bool RESTRICT, int NC>
__global__ __launch_bounds__(1024) void k_single_block3(LV<T> L, LV<T> Lc, int steps, int into_old) {
    constexpr int N = 16, NH = 8, NT = 1024, H = N / 2;
    using B = Blk<3, N>;
    using CT = ColTile<N>;
    constexpr int PER = B::HALF / NT;
    constexpr int TS = 2 * CT::SIZE, NAT = RESTRICT ? 2 * B::CPB : 0;
    __shared__ T sm[TS > NAT ? TS : NAT];
    __shared__ T sbv[2 * 5 * 256];
    T *tile[2] = {sm, sm + CT::SIZE};
    const int rhs = rhs_of(L), t = threadIdx.x;
    const int leaf = L.leaf[0];
    const int4 P = L.pos[0];
    const int mo = L.map_off ? L.map_off[0] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    int nbk[6] = {-2, -2, -2, -2, -2, -2};
    tables_loaded(act, leaf, P, nbk, mo);
    if (!act) return;
    const bool fas = FAS && !leaf;
    T *phi = L.phi + (long long)rhs * L.fstride;
    T *g = L.g + (long long)rhs * L.fstride;
    const T *src = FAS ? L.old + (long long)rhs * L.fstride : phi;
    T val[2][PER], gv[2][PER], rc[2][PER][8], bt[2][PER];
    int ri[2][PER];
#pragma unroll
    for (int c = 0; c < 2; c++) {
        load_cells<T, PER, NT, true>(src + c * B::HALF, t, val[c]);
        load_cells<T, PER, NT, true>(g + c * B::HALF, t, gv[c]);
#pragma unroll
        for (int m = 0; m < PER; m++) ri[c][m] = mo >= 0 ? L.map[mo + c * B::HALF + cell_of<NT, true>(t, m)] : -1;
    }
    // face values of the Dirichlet ghosts, per reading colour u (the cell
    // indices of stage_colour's face entries)
    if (t < N * N) {
#pragma unroll
        for (int u = 0; u < 2; u++) {
            T *bvu = sbv + u * 5 * 256;
            auto face = [&](int d, int i, int j, int k) -> T {
                const int ax = d >> 1, sd = (d & 1) ? 1 : -1;
                return !zero_flux(L.neumann, ax, sd) && L.bcv
                           ? L.bcv[face_slot<3>(ax, sd, P.x * N + i, P.y * N + j, P.z * N + k, L.n, L.nface)]
                           : T(0);
            };
            if (t < N * NH) {
                const int fh = t % NH, fr = t / NH;
                bvu[t] = face(2, 2 * fh + ((u + fr) & 1), 0, fr);
                bvu[256 + t] = face(3, 2 * fh + ((u + N - 1 + fr) & 1), N - 1, fr);
                bvu[512 + t] = face(4, 2 * fh + ((u + fr) & 1), fr, 0);
                bvu[768 + t] = face(5, 2 * fh + ((u + fr + N - 1) & 1), fr, N - 1);
            }
            const int xj = t % N, xk = t / N, xp = (u + xj + xk) & 1;
            bvu[1024 + t] = face(xp, xp ? N - 1 : 0, xj, xk);
        }
    }
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int m = 0; m < PER; m++) {
#pragma unroll
            for (int d = 0; d < 8; d++) rc[c][m][d] = T(0);
            bt[c][m] = T(0);
            if (ri[c][m] >= 0) {
                const T *r = L.rec + 8 * (long long)ri[c][m];
#pragma unroll
                for (int d = 0; d < 8; d++) rc[c][m][d] = r[d];
                if (L.b) bt[c][m] = L.b[ri[c][m]];
            }
        }
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int q = cell_of<NT, true>(t, m);
            tile[c][CT::at(q / (NH * N), (q / NH) % N, q % NH)] = val[c][m];
        }
    __syncthreads();
    sb_ghosts<T>(tile[1], tile[0], sbv, 0, L.neumann, t);
    sb_ghosts<T>(tile[0], tile[1], sbv + 5 * 256, 1, L.neumann, t);
    __syncthreads();
    // L phi at the thread's cells of colour c (tile_op's arithmetic)
    auto apply_op = [&](int c, T *out) {
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int q = cell_of<NT, true>(t, m);
            int i, j, k;
            T v[6];
            tile_neighbours<T, N>(tile[1 - c], c, q, i, j, k, v);
            const T own = tile[c][CT::at(k, j, q % NH)];
            if (ri[c][m] < 0) {
                out[m] = L.inv_dx2 * ((((v[0] + v[1]) + (v[2] + v[3])) + (v[4] + v[5])) - T(6) * own);
            } else {
                T s = T(0);
#pragma unroll
                for (int d = 0; d < 6; d++) s += rc[c][m][d] * v[d];
                out[m] = s + rc[c][m][6] * own + bt[c][m];
            }
        }
    };
    if (fas) {
        // FAS right-hand side g = L old + g (the restricted residual)
#pragma unroll
        for (int c = 0; c < 2; c++) {
            T lp[PER];
            apply_op(c, lp);
#pragma unroll
            for (int m = 0; m < PER; m++) gv[c][m] = lp[m] + gv[c][m];
            store_cells<T, PER, NT, true>(g + c * B::HALF, t, gv[c]);
        }
        __syncthreads();  // the first half sweep writes the tile read here
    }
    const T inv6 = T(1) / T(6);
    for (int st = 0; st < steps; st++) {
#pragma unroll
        for (int u = 0; u < 2; u++) {
            // half sweep of colour u (gs_half3_body's arithmetic), and the
            // ghosts the other colour will read, from colour 1-u, which this
            // half sweep does not change
#pragma unroll
            for (int m = 0; m < PER; m++) {
                const int q = cell_of<NT, true>(t, m);
                int i, j, k;
                T v[6];
                tile_neighbours<T, N>(tile[1 - u], u, q, i, j, k, v);
                T nv;
                if (ri[u][m] < 0) {
                    nv = (((v[0] + v[1]) + (v[2] + v[3])) + (v[4] + v[5]) - L.dx2 * gv[u][m]) * inv6;
                } else {
                    T s = T(0);
#pragma unroll
                    for (int d = 0; d < 6; d++) s += rc[u][m][d] * v[d];
                    nv = (gv[u][m] - bt[u][m] - s) * rc[u][m][7];
                }
                tile[u][CT::at(k, j, q % NH)] = nv;
            }
            sb_ghosts<T>(tile[u], tile[1 - u], sbv + (1 - u) * 5 * 256, 1 - u, L.neumann, t);
            __syncthreads();
        }
    }
    T own[2][PER];
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int q = cell_of<NT, true>(t, m);
            own[c][m] = tile[c][CT::at(q / (NH * N), (q / NH) % N, q % NH)];
        }
    if (FAS || steps > 0)
#pragma unroll
        for (int c = 0; c < 2; c++) store_cells<T, PER, NT, true>(phi + c * B::HALF, t, own[c]);
    if (!RESTRICT) return;
    // residual g - L phi from the final iterate: the ghosts of colour 0's
    // tile still hold colour 1's values from before its last half sweep
    if (steps > 0) {
        sb_ghosts<T>(tile[0], tile[1], sbv + 5 * 256, 1, L.neumann, t);
        __syncthreads();
    }
    T r[2][PER];
#pragma unroll
    for (int c = 0; c < 2; c++) {
        apply_op(c, r[c]);
#pragma unroll
        for (int m = 0; m < PER; m++) r[c][m] = gv[c][m] - r[c][m];
    }
    __syncthreads();  // the tiles become the natural-order arrays of r and phi
    T *sr = sm, *sp = sm + B::CPB;
#pragma unroll
    for (int c = 0; c < 2; c++)
#pragma unroll
        for (int m = 0; m < PER; m++) {
            int i, j, k;
            q_to_ijk<N>(c, cell_of<NT, true>(t, m), i, j, k);
            sr[(k * N + j) * N + i] = r[c][m];
            sp[(k * N + j) * N + i] = own[c][m];
        }
    __syncthreads();
    if (t >= H * H * H) return;
    const int ci = t % H, cj = (t / H) % H, ck = t / (H * H);
    T rs = T(0), ps = T(0);
#pragma unroll
    for (int ch = 0; ch < 8; ch++) {
        const int e = ((2 * ck + ((ch >> 2) & 1)) * N + 2 * cj + ((ch >> 1) & 1)) * N + 2 * ci + (ch & 1);
        rs += sr[e];
        ps += sp[e];
    }
    const int C0[3] = {P.x * H, P.y * H, P.z * H};
    const int pb = block_at<T, 3>(Lc, C0[0] / NC, C0[1] / NC, C0[2] / NC);
    if (pb < 0) return;  // excluded by construction: every block has a parent
    const T inv = T(0.125);
    const int gi = C0[0] + ci, gj = C0[1] + cj, gk = C0[2] + ck;
    const long long o = (long long)rhs * Lc.fstride + (long long)pb * Blk<3, NC>::CPB +
                        split_of<3, NC>(gi % NC, gj % NC, gk % NC);
    const T pv = ps * inv;
    Lc.old[o] = pv;
    if (!into_old) Lc.phi[o] = pv;
    Lc.g[o] = rs * inv;
}

// LATE as in the restriction
template <typename T, int N, int NTC, bool LATE>
__global__ __launch_bounds__(2 * NTC) __attribute__((amdgpu_waves_per_eu(LATE ? 6 : 1))) void k_residual_max3_pair(
    LV<T> L, LV<T> Lc, unsigned long long *out) {
    using B = Blk<3, N>;
    constexpr int PER = B::HALF / NTC;
    constexpr bool V2 = cell_pairs<N>();
    __shared__ T tiles[PairTiles<T, N>::SIZE];
    __shared__ double wmax[2 * NTC / 64];
    const int blk = block_of(L), rhs = rhs_of(L);
    const int c = threadIdx.x / NTC, t = threadIdx.x % NTC;
    const int leaf = L.leaf[blk];
    const int4 P = L.pos[blk];
    int nbk[6];
    face_ids<T, N>(L, blk, nbk);
    const int mo = L.map_off ? L.map_off[blk] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    tables_loaded(act, leaf, P, nbk, mo);
    if (!act || !leaf) return;
    const T *__restrict__ phi = L.phi + (long long)rhs * L.fstride;
    const T *__restrict__ g = L.g + (long long)rhs * L.fstride;
    const T *phic = Lc.phi ? Lc.phi + (long long)rhs * Lc.fstride : nullptr;
    const long long base = (long long)blk * B::CPB + c * B::HALF;
    T own[PER], lp[PER], gv[PER];
    int ri[PER];
    load_cells<T, PER, NTC, V2>(phi + base, t, own);
    if (!LATE) load_cells<T, PER, NTC, V2>(g + base, t, gv);
#pragma unroll
    for (int m = 0; m < PER; m++) ri[m] = mo >= 0 ? L.map[mo + c * B::HALF + cell_of<NTC, V2>(t, m)] : -1;
    pair_op<T, N, NTC, LATE>(L, Lc, phi, phic, tiles, blk, nbk, P, ri, own, lp);
    if (LATE) load_cells<T, PER, NTC, V2>(g + base, t, gv);
    double mx = 0.0;
#pragma unroll
    for (int m = 0; m < PER; m++) mx = fmax(mx, abs_nan_inf((double)(gv[m] - lp[m])));
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    if (threadIdx.x % 64 == 0) wmax[threadIdx.x / 64] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 2 * NTC / 64; w++) mx = fmax(mx, wmax[w]);
        if (mx != mx) mx = __longlong_as_double(0x7ff0000000000000ll);
        atomicMax(norm_slot(out, rhs), (unsigned long long)__double_as_longlong(mx));
    }
}

// max |g - L phi| over a leaf block (3D); ZERO: residual of phi = 0
template <typename T, int N, bool ZERO>
__global__ __launch_bounds__(256) void k_residual_max3(LV<T> L, LV<T> Lc, unsigned long long *out) {
    using B = Blk<3, N>;
    constexpr int PER = Per<N>::PER;
    const int blk = block_of(L);
    const int rhs = rhs_of(L);
    const int leaf = L.leaf[blk];
    const int4 P = L.pos[blk];
    int nbk[6];
    face_ids<T, N>(L, blk, nbk);
    const int mo = L.map_off ? L.map_off[blk] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    tables_loaded(act, leaf, P, nbk, mo);
    if (!act || !leaf) return;
    __shared__ T tile[ColTile<N>::SIZE];
    __shared__ double wmax[4];
    const T *__restrict__ phi = L.phi + (long long)rhs * L.fstride;
    const T *__restrict__ g = L.g + (long long)rhs * L.fstride;
    const T *phic = Lc.phi ? Lc.phi + (long long)rhs * Lc.fstride : nullptr;
    const long long base = (long long)blk * B::CPB;
    T own0[PER], own1[PER], lp[PER], gv[PER];
    int ri[PER];
    double mx = 0.0;
#pragma unroll
    for (int c = 0; c < 2; c++) {
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int s = c * B::HALF + threadIdx.x + 256 * m;
            if (c == 0) own0[m] = ZERO ? T(0) : phi[base + s];
            gv[m] = g[base + s];
            ri[m] = mo >= 0 ? L.map[mo + s] : -1;
        }
        colour_pass<T, N, ZERO>(L, Lc, phi, phic, tile, blk, nbk, P, ri, c, c == 0 ? own0 : own1,
                                c == 0 || ZERO ? nullptr : own0, lp);
        if (c == 0) {
            if (ZERO) {
#pragma unroll
                for (int m = 0; m < PER; m++) own1[m] = T(0);
            } else {
                own_from_tile<T, N>(tile, own1);
            }
        }
#pragma unroll
        for (int m = 0; m < PER; m++) mx = fmax(mx, abs_nan_inf((double)(gv[m] - lp[m])));
        __syncthreads();
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    if (threadIdx.x % 64 == 0) wmax[threadIdx.x / 64] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; w++) mx = fmax(mx, wmax[w]);
        if (mx != mx) mx = __longlong_as_double(0x7ff0000000000000ll);
        atomicMax(norm_slot(out, rhs), (unsigned long long)__double_as_longlong(mx));
    }
}

// prolongation, 3D: the coarse correction of the parent region (plus a
// one-cell halo) is staged in LDS, then every fine cell is updated once.
// NT threads per workgroup; all coarse loads of a thread are issued before
// its LDS writes.
template <typename T, int N, int NC, bool SOL, int NT>
__device__ __forceinline__ void prolong3_body(const LV<T> &L, const LV<T> &Lc, int blk, int rhs, T *et) {
    using B = Blk<3, N>;
    constexpr int H = N / 2, E = H + 2, ESZ = E * E * E, PER = B::CPB / NT, EPER = (ESZ + NT - 1) / NT;
    constexpr bool V2 = cell_pairs<N>();
    const int4 P = L.pos[blk];
    const int act = L.active ? L.active[rhs] : 1;
    asm volatile("" ::"s"(act), "s"(P.x), "s"(P.y), "s"(P.z));  // both loads in one round trip
    if (!act) return;
    const T *phic = Lc.phi + (long long)rhs * Lc.fstride;
    const T *oldc = Lc.old + (long long)rhs * Lc.fstride;
    T *__restrict__ phi = L.phi + (long long)rhs * L.fstride + (long long)blk * B::CPB;
    T f[PER];
    load_cells<T, PER, NT, V2>(phi, threadIdx.x, f);
    const int C0[3] = {P.x * H, P.y * H, P.z * H};
    T ev[EPER];
#pragma unroll
    for (int m = 0; m < EPER; m++) {
        const int e = threadIdx.x + NT * m;
        if (e < ESZ) {
            const int x = e % E, y = (e / E) % E, z = e / (E * E);
            ev[m] = coarse_e<T, 3, NC, SOL>(Lc, phic, oldc, C0[0] + x - 1, C0[1] + y - 1, C0[2] + z - 1);
        }
    }
#pragma unroll
    for (int m = 0; m < EPER; m++) {
        const int e = threadIdx.x + NT * m;
        if (e < ESZ) et[e] = ev[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PER; m++) {
        const int s = cell_of<NT, V2>(threadIdx.x, m);
        int i, j, k;
        q_to_ijk<N>(s / B::HALF, s % B::HALF, i, j, k);
        const int ci = (i >> 1) + 1, cj = (j >> 1) + 1, ck = (k >> 1) + 1;
        const int ox = (i & 1) ? 1 : -1, oy = (j & 1) ? 1 : -1, oz = (k & 1) ? 1 : -1;
        T e = T(0);
#pragma unroll
        for (int dl = 0; dl < 8; dl++) {
            const int ax = dl & 1, ay = (dl >> 1) & 1, az = (dl >> 2) & 1;
            const T w = (ax ? T(0.25) : T(0.75)) * (ay ? T(0.25) : T(0.75)) * (az ? T(0.25) : T(0.75));
            e = e + w * et[((ck + az * oz) * E + (cj + ay * oy)) * E + (ci + ax * ox)];
        }
        f[m] = f[m] + e;
    }
    store_cells<T, PER, NT, V2>(phi, threadIdx.x, f);
}

template <typename T, int N, int NC, bool SOL, int NT>
__global__ __launch_bounds__(NT) void k_prolong3(LV<T> L, LV<T> Lc) {
    constexpr int H = N / 2, E = H + 2, ESZ = E * E * E;
    __shared__ T et[ESZ];
    prolong3_body<T, N, NC, SOL, NT>(L, Lc, block_of(L), rhs_of(L), et);
}

// Prolongation of the coarse correction (as k_prolong3) fused with the red
// half sweep that follows it (as k_gs_half3, colour 0), 3D.  The red cells'
// prolonged values are only read where a cell forms its own ghost (domain
// and refinement faces), and the black cells' prolonged values only by this
// half sweep (as neighbours, the face halo included: the fine cells just
// outside the block interpolate from the block's one-cell coarse halo) and
// by the next black half sweep, for its own ghosts.  So the black values
// are prolonged in LDS and not stored in phi (the next black half sweep
// overwrites them); blocks with a domain or refinement face store them in
// L.own, from where that black half sweep takes its own values.  Every
// value is formed with the same operations in the same order as by the two
// separate kernels.
template <typename T, int N>
__device__ __forceinline__ T prolonged(const T *et, int i, int j, int k) {
    constexpr int E = N / 2 + 2;
    const int ci = (i >> 1) + 1, cj = (j >> 1) + 1, ck = (k >> 1) + 1;
    const int ox = (i & 1) ? 1 : -1, oy = (j & 1) ? 1 : -1, oz = (k & 1) ? 1 : -1;
    T e = T(0);
#pragma unroll
    for (int dl = 0; dl < 8; dl++) {
        const int ax = dl & 1, ay = (dl >> 1) & 1, az = (dl >> 2) & 1;
        const T w = (ax ? T(0.25) : T(0.75)) * (ay ? T(0.25) : T(0.75)) * (az ? T(0.25) : T(0.75));
        e = e + w * et[((ck + az * oz) * E + (cj + ay * oy)) * E + (ci + ax * ox)];
    }
    return e;
}

template <typename T, int N, int NC, int NT, bool V2>
__device__ __forceinline__ void prolong_gs3_body(const LV<T> &L, const LV<T> &Lc, int blk, int rhs, T *tile, T *et,
                                                 T *rp) {
    using B = Blk<3, N>;
    using CT = ColTile<N>;
    constexpr int NH = N / 2, H = N / 2, E = H + 2, ESZ = E * E * E, PER = B::HALF / NT,
                  EPER = (ESZ + NT - 1) / NT;
    const int4 P = L.pos[blk];
    int nbk[6];
    face_ids<T, N>(L, blk, nbk);
    const int mo = L.map_off ? L.map_off[blk] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    tables_loaded(act, 1, P, nbk, mo);
    if (!act) return;
    bool ghosts = false;  // a domain or refinement face: cells form ghosts from their own values
#pragma unroll
    for (int d = 0; d < 6; d++) ghosts |= nbk[d] < 0;
    T *__restrict__ phi = L.phi + (long long)rhs * L.fstride;
    const long long base = (long long)blk * B::CPB;
    const T *phic = Lc.phi + (long long)rhs * Lc.fstride;
    const T *oldc = Lc.old + (long long)rhs * Lc.fstride;
    const int t = threadIdx.x;
    // loads: the coarse correction with its one-cell halo, the red cells'
    // values where ghosts need them (g of the red cells and their record
    // rows are loaded after the prolongation, which keeps them out of the
    // registers live across it)
    T gv[PER], ro[PER];
    int ri[PER];
    const int C0[3] = {P.x * H, P.y * H, P.z * H};
    T ev[EPER];
#pragma unroll
    for (int m = 0; m < EPER; m++) {
        const int e = t + NT * m;
        if (e < ESZ) {
            const int x = e % E, y = (e / E) % E, z = e / (E * E);
            ev[m] = coarse_e<T, 3, NC, false>(Lc, phic, oldc, C0[0] + x - 1, C0[1] + y - 1, C0[2] + z - 1);
        }
    }
    if (ghosts) load_cells<T, PER, NT, V2>(phi + base, t, ro);
    // without ghosts the black colour and its halos are staged right away
    // (their loads overlap the coarse ones); the own values are never read
    if (!ghosts) stage_colour<T, N, false, NT, V2>(tile, L, phi, blk, nbk, P, 1, t);
#pragma unroll
    for (int m = 0; m < EPER; m++) {
        const int e = t + NT * m;
        if (e < ESZ) et[e] = ev[m];
    }
    __syncthreads();
    if (ghosts) {
        // prolonged red values, then the black colour staged with the domain
        // ghosts of the red cells formed from them
#pragma unroll
        for (int m = 0; m < PER; m++) {
            int i, j, k;
            const int q = cell_of<NT, V2>(t, m);
            q_to_ijk<N>(0, q, i, j, k);
            rp[q] = ro[m] + prolonged<T, N>(et, i, j, k);
        }
        __syncthreads();
        stage_colour<T, N, false, NT, V2>(tile, L, phi, blk, nbk, P, 1, t, nullptr, rp);
        __syncthreads();
    }
    // prolong the staged black values: the block's cells and the halo cells
    // of same-level neighbours (domain ghosts are final; refinement-face
    // slots are filled below)
#pragma unroll
    for (int m = 0; m < PER; m++) {
        int i, j, k;
        const int q = cell_of<NT, V2>(t, m);
        q_to_ijk<N>(1, q, i, j, k);
        const int a = CT::at(k, j, q % NH);
        tile[a] = tile[a] + prolonged<T, N>(et, i, j, k);
    }
    {
        const int fh = t % NH, fr = t / NH;  // y/z face entries, as in stage_colour
        if (t < N * NH) {
            const int k = fr, jz = fr;
            if (nbk[2] >= 0) {
                const int a = CT::at(k, -1, fh);
                tile[a] = tile[a] + prolonged<T, N>(et, 2 * fh + (k & 1), -1, k);
            }
            if (nbk[3] >= 0) {
                const int a = CT::at(k, N, fh);
                tile[a] = tile[a] + prolonged<T, N>(et, 2 * fh + ((N - 1 + k) & 1), N, k);
            }
            if (nbk[4] >= 0) {
                const int a = CT::at(-1, jz, fh);
                tile[a] = tile[a] + prolonged<T, N>(et, 2 * fh + (jz & 1), jz, -1);
            }
            if (nbk[5] >= 0) {
                const int a = CT::at(N, jz, fh);
                tile[a] = tile[a] + prolonged<T, N>(et, 2 * fh + ((jz + N - 1) & 1), jz, N);
            }
        }
        const int xj = t % N, xk = t / N;  // x face entries
        if (t < N * N) {
            const int xp = (xj + xk) & 1, nbx = xp ? nbk[1] : nbk[0];
            if (nbx >= 0) {
                const int a = CT::at(xk, xj, xp ? NH : -1);
                tile[a] = tile[a] + prolonged<T, N>(et, xp ? N : -1, xj, xk);
            }
        }
    }
    // (non-temporal in FP64 only, as in the sweep)
    load_cells<T, PER, NT, V2, sizeof(T) == 8>(L.g + (long long)rhs * L.fstride + base, t, gv);
#pragma unroll
    for (int m = 0; m < PER; m++) ri[m] = mo >= 0 ? L.map[mo + cell_of<NT, V2>(t, m)] : -1;
    __syncthreads();
    if (any_coarser(nbk)) {
        coarser_face_ghosts<T, N, NT>(tile, Lc, rp, phic, nbk, P, 0, t);
        __syncthreads();
    }
    // the red half sweep on the prolonged black values
    const T inv6 = T(1) / T(6);
    T nv[PER];
#pragma unroll
    for (int m = 0; m < PER; m++) {
        const int q = cell_of<NT, V2>(t, m);
        int i, j, k;
        T v[6];
        tile_neighbours<T, N>(tile, 0, q, i, j, k, v);
        if (ri[m] < 0) {
            nv[m] = (((v[0] + v[1]) + (v[2] + v[3])) + (v[4] + v[5]) - L.dx2 * gv[m]) * inv6;
        } else {
            const T *r = L.rec + 8 * (long long)ri[m];
            T sum = T(0);
#pragma unroll
            for (int d = 0; d < 6; d++) sum += r[d] * v[d];
            const T bt = L.b ? L.b[ri[m]] : T(0);
            nv[m] = (gv[m] - bt - sum) * r[7];
        }
    }
    store_cells<T, PER, NT, V2>(phi + base, t, nv);
    if (ghosts) {  // prolonged black values for the next black half sweep's ghosts
        T bv[PER];
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int q = cell_of<NT, V2>(t, m);
            bv[m] = tile[CT::at(q / (NH * N), (q / NH) % N, q % NH)];
        }
        store_cells<T, PER, NT, V2>(L.own + (long long)rhs * L.fstride + base + B::HALF, t, bv);
    }
}

// 512 threads: at most 80 VGPRs, three workgroups per CU (LDS allows three)
template <typename T, int N, int NC, int NT, bool V2>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 512 ? 6 : 1))) void k_prolong_gs3(LV<T> L,
                                                                                                           LV<T> Lc) {
    constexpr int E = N / 2 + 2;
    __shared__ T tile[ColTile<N>::SIZE];
    __shared__ T et[E * E * E];
    __shared__ T rp[Blk<3, N>::HALF];
    prolong_gs3_body<T, N, NC, NT, V2>(L, Lc, block_of(L), rhs_of(L), tile, et, rp);
}

// The FP32 correction's first red half sweep when the correction is zero
// everywhere (every neighbour and ghost value is +0): the arithmetic of
// gs_half3_body with those zeros, so the value is the same bits.  r32: the
// cell's FP32 right-hand side; ri its record (-1: standard stencil).
__device__ __forceinline__ float zero_start_red(const LV<float> &L32, float r32, int ri) {
    if (ri < 0) {
        const float inv6 = 1.0f / 6.0f;
        return (0.0f - L32.dx2 * r32) * inv6;
    }
    return r32 * L32.rec[8 * (long long)ri + 7];
}

// mixed precision defect (FP64): g32 = g - L phi on a leaf block, phi32 = 0,
// or with red_preset the red cells' phi32 after the correction's first red
// half sweep from zero (zero_start_red)
template <int N>
__global__ __launch_bounds__(256) void k_defect3(LV<double> L, LV<double> Lc, LV<float> L32, const int *lb,
                                                  unsigned long long *out, int red_preset) {
    using B = Blk<3, N>;
    constexpr int PER = Per<N>::PER;
    __shared__ double tile[ColTile<N>::SIZE];
    __shared__ double wmax[4];
    const int rhs = rhs_of(L);
    const int blk = lb[leaf_slot(L)];
    const int4 P = L.pos[blk];
    int nbk[6];
    face_ids<double, N>(L, blk, nbk);
    const int mo = L.map_off ? L.map_off[blk] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    tables_loaded(act, 1, P, nbk, mo);
    if (!act) return;
    const double *__restrict__ phi = L.phi + (long long)rhs * L.fstride;
    const double *__restrict__ g = L.g + (long long)rhs * L.fstride;
    const double *phic = Lc.phi ? Lc.phi + (long long)rhs * Lc.fstride : nullptr;
    const long long base = (long long)blk * B::CPB;
    float *g32 = L32.g + (long long)rhs * L32.fstride + base;
    float *p32 = L32.phi + (long long)rhs * L32.fstride + base;
    double own0[PER], own1[PER], lp[PER], gv[PER];
    int ri[PER];
    double mx = 0.0;
#pragma unroll
    for (int c = 0; c < 2; c++) {
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int s = c * B::HALF + threadIdx.x + 256 * m;
            if (c == 0) own0[m] = phi[base + s];
            gv[m] = g[base + s];
            ri[m] = mo >= 0 ? L.map[mo + s] : -1;
        }
        colour_pass<double, N, false>(L, Lc, phi, phic, tile, blk, nbk, P, ri, c, c == 0 ? own0 : own1,
                                      c == 0 ? nullptr : own0, lp);
        if (c == 0) own_from_tile<double, N>(tile, own1);
#pragma unroll
        for (int m = 0; m < PER; m++) {
            const int s = c * B::HALF + threadIdx.x + 256 * m;
            const double r = gv[m] - lp[m];
            mx = fmax(mx, abs_nan_inf(r));
            g32[s] = (float)r;
            p32[s] = red_preset && c == 0 ? zero_start_red(L32, (float)r, ri[m]) : 0.0f;
        }
        __syncthreads();
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    if (threadIdx.x % 64 == 0) wmax[threadIdx.x / 64] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; w++) mx = fmax(mx, wmax[w]);
        if (mx != mx) mx = __longlong_as_double(0x7ff0000000000000ll);
        atomicMax(norm_slot(out, rhs), (unsigned long long)__double_as_longlong(mx));
    }
}

// the same defect with both colours staged at once by two wave groups (the
// residual arithmetic of k_residual_max3_pair, the same bits as k_defect3);
// LATE as in the restriction
template <int N, int NTC, bool LATE>
__global__ __launch_bounds__(2 * NTC) __attribute__((amdgpu_waves_per_eu(LATE ? 6 : 1))) void k_defect3_pair(
    LV<double> L, LV<double> Lc, LV<float> L32, const int *lb, unsigned long long *out, int red_preset) {
    using B = Blk<3, N>;
    constexpr int PER = B::HALF / NTC;
    constexpr bool V2 = cell_pairs<N>();
    __shared__ double tiles[PairTiles<double, N>::SIZE];
    __shared__ double wmax[2 * NTC / 64];
    const int rhs = rhs_of(L);
    const int blk = lb[leaf_slot(L)];
    const int c = threadIdx.x / NTC, t = threadIdx.x % NTC;
    const int4 P = L.pos[blk];
    int nbk[6];
    face_ids<double, N>(L, blk, nbk);
    const int mo = L.map_off ? L.map_off[blk] : -1;
    const int act = L.active ? L.active[rhs] : 1;
    tables_loaded(act, 1, P, nbk, mo);
    if (!act) return;
    const double *__restrict__ phi = L.phi + (long long)rhs * L.fstride;
    const double *__restrict__ g = L.g + (long long)rhs * L.fstride;
    const double *phic = Lc.phi ? Lc.phi + (long long)rhs * Lc.fstride : nullptr;
    const long long base = (long long)blk * B::CPB + c * B::HALF;
    float *g32 = L32.g + (long long)rhs * L32.fstride + base;
    float *p32 = L32.phi + (long long)rhs * L32.fstride + base;
    double own[PER], lp[PER], gv[PER];
    int ri[PER];
    load_cells<double, PER, NTC, V2>(phi + base, t, own);
    // g with the non-temporal hint: 99.8 -> 93.9 us at 256^3.  The FP64
    // residual and restriction keep plain loads: with the hint they ran 3 us
    // faster, but the sweeps after them, which find those g lines cached,
    // 0.8-2.4 us slower
    if (!LATE) load_cells<double, PER, NTC, V2, true>(g + base, t, gv);
#pragma unroll
    for (int m = 0; m < PER; m++) ri[m] = mo >= 0 ? L.map[mo + c * B::HALF + cell_of<NTC, V2>(t, m)] : -1;
    pair_op<double, N, NTC, LATE>(L, Lc, phi, phic, tiles, blk, nbk, P, ri, own, lp);
    if (LATE) load_cells<double, PER, NTC, V2, true>(g + base, t, gv);
    float r32[PER], z32[PER];
    double mx = 0.0;
#pragma unroll
    for (int m = 0; m < PER; m++) {
        const double r = gv[m] - lp[m];
        mx = fmax(mx, abs_nan_inf(r));
        r32[m] = (float)r;
        z32[m] = red_preset && c == 0 ? zero_start_red(L32, r32[m], ri[m]) : 0.0f;
    }
    store_cells<float, PER, NTC, V2>(g32, t, r32);
    store_cells<float, PER, NTC, V2>(p32, t, z32);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    if (threadIdx.x % 64 == 0) wmax[threadIdx.x / 64] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 2 * NTC / 64; w++) mx = fmax(mx, wmax[w]);
        if (mx != mx) mx = __longlong_as_double(0x7ff0000000000000ll);
        atomicMax(norm_slot(out, rhs), (unsigned long long)__double_as_longlong(mx));
    }
}

// ================================================ bottom of the V-cycle, fused
// Levels with few blocks are launch- and latency-bound: one launch costs a
// few microseconds even for a single workgroup.  k_small_vcycle runs the
// V-cycle below and including level `top` (smoothing, FAS restriction,
// coarse solve, prolongation) in one cooperative launch.  Each phase is a
// loop of the workgroups over (block, rhs) items calling the same per-block
// bodies as the standalone kernels, followed by a grid-wide barrier, so the
// results are identical to the launch-per-phase path.

__device__ __forceinline__ void copy_parents_body3(int N, const LV<double> &L, int blk, int rhs) {
    if (L.active && !L.active[rhs]) return;
    const int cpb = N * N * N;
    const long long o = (long long)rhs * L.fstride + (long long)blk * cpb;
    if (L.leaf[blk]) {
        for (int c = threadIdx.x; c < cpb; c += blockDim.x) L.old[o + c] = L.phi[o + c];
        return;
    }
    for (int c = threadIdx.x; c < cpb; c += blockDim.x) L.phi[o + c] = L.old[o + c];
}
__device__ __forceinline__ void copy_parents_body3(int N, const LV<float> &L, int blk, int rhs) {
    if (L.active && !L.active[rhs]) return;
    const int cpb = N * N * N;
    const long long o = (long long)rhs * L.fstride + (long long)blk * cpb;
    if (L.leaf[blk]) {
        for (int c = threadIdx.x; c < cpb; c += blockDim.x) L.old[o + c] = L.phi[o + c];
        return;
    }
    for (int c = threadIdx.x; c < cpb; c += blockDim.x) L.phi[o + c] = L.old[o + c];
}

// exact coarse solve, rows [tile*32, tile*32+32) of one rhs (3D, 8^3 grid)
template <typename T>
__device__ __forceinline__ void coarse_solve3_body(const LV<T> &L0, const double *M, const double *S, int tile, int rhs,
                                                   double *rhsv) {
    constexpr int NB = 8, NCELL = 512, ROWS = 32;
    if (L0.active && !L0.active[rhs]) return;
    const T *g = L0.g + (long long)rhs * L0.fstride;
    T *phi = L0.phi + (long long)rhs * L0.fstride;
    const int mo = L0.map_off ? L0.map_off[0] : -1;
    const double inv = 1.0 / ((double)L0.dx2);
    for (int c = threadIdx.x; c < NCELL; c += blockDim.x) {
        const int i = c % NB, j = (c / NB) % NB, k = c / (NB * NB);
        const int si = split_of<3, NB>(i, j, k);
        const int ri = mo >= 0 ? L0.map[mo + si] : -1;
        double r = (double)g[si];
        if (ri >= 0 && L0.b) r -= (double)L0.b[ri];
        for (int d = 0; d < 6; d++) {
            const int ax = d >> 1, s = (d & 1) ? 1 : -1;
            int q[3] = {i, j, k};
            q[ax] += s;
            if (q[ax] >= 0 && q[ax] < NB) continue;
            const double cc = ri >= 0 ? (double)L0.rec[8 * (long long)ri + d] : inv;
            if (cc == 0.0 || zero_flux(L0.neumann, ax, s)) continue;  // zero flux: folded into the operator
            const double bv = L0.bcv ? (double)L0.bcv[face_slot<3>(ax, s, i, j, k, NB, L0.nface)] : 0.0;
            r -= 2.0 * cc * bv;
        }
        rhsv[c] = S[c] * r;
    }
    __syncthreads();
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int row = tile * ROWS + wave; row < (tile + 1) * ROWS; row += blockDim.x / 64) {
        double acc = 0.0;
        for (int c = lane; c < NCELL; c += 64) acc += M[(long long)row * NCELL + c] * rhsv[c];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lane == 0) {
            const int i = row % NB, j = (row / NB) % NB, k = row / (NB * NB);
            phi[split_of<3, NB>(i, j, k)] = (T)acc;
        }
    }
}

// out-of-line entry points of the per-block bodies for the fused kernel: each
// keeps its own register allocation instead of the fused kernel taking the
// union of all of them
template <typename T, int N>
__device__ __noinline__ void gs_call(const LV<T> &L, const LV<T> &Lc, int color, int blk, int rhs, T *sm) {
    gs_half3_body<T, N>(L, Lc, color, blk, rhs, sm);
}
template <typename T, int N, int NC>
__device__ __noinline__ void restrict_call(const LV<T> &L, const LV<T> &Lc, int into_old, int blk, int rhs, T *sm) {
    restrict_fas3_body<T, N, NC>(L, Lc, into_old, blk, rhs, sm);
}
template <typename T, int N>
__device__ __noinline__ void fas_rhs_call(const LV<T> &L, const LV<T> &Lc, int blk, int rhs, T *sm) {
    fas_rhs3_body<T, N>(L, Lc, 1, blk, rhs, sm);
}
template <typename T, int N, int NC>
__device__ __noinline__ void prolong_call(const LV<T> &L, const LV<T> &Lc, int blk, int rhs, T *sm) {
    prolong3_body<T, N, NC, false, 256>(L, Lc, blk, rhs, sm);
}
template <typename T>
__device__ __noinline__ void coarse_call(const LV<T> &L0, const double *M, const double *S, int tile, int rhs,
                                         double *sm) {
    coarse_solve3_body<T>(L0, M, S, tile, rhs, sm);
}

template <typename T>
__global__ __launch_bounds__(256) void k_small_vcycle(const SmallLevels<T> *__restrict__ P, int top) {
    __shared__ double smem[4096];  // largest body: restriction of a 16^3 block (32 KB)
    T *sm = reinterpret_cast<T *>(smem);
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    const int G = gridDim.x, R = P->nrhs, into_old = P->into_old;
#define OCTMG_PHASE(NBLK, ...)                                                  \
    {                                                                           \
        const int nb_ = (NBLK);                                                 \
        for (int it_ = blockIdx.x; it_ < nb_ * R; it_ += G) {                   \
            const int blk = it_ % nb_, rhs = it_ / nb_;                         \
            __VA_ARGS__;                                                        \
            __syncthreads();                                                    \
        }                                                                       \
        grid.sync();                                                            \
    }
    for (int il = top; il > 0; il--) {
        const LV<T> &L = P->L[il], &Lc = P->L[il - 1];
        const LV<T> &Lcc = P->L[il >= 2 ? il - 2 : il - 1];
        const int N = P->N[il], NC = P->N[il - 1];
        for (int st = 0; st < P->n_down; st++)
            for (int color = 0; color < 2; color++)
                OCTMG_PHASE(L.nblocks, if (N == 16) gs_call<T, 16>(L, Lc, color, blk, rhs, sm);
                            else gs_call<T, 8>(L, Lc, color, blk, rhs, sm))
        OCTMG_PHASE(L.nblocks, if (N == 16 && NC == 16) restrict_call<T, 16, 16>(L, Lc, into_old, blk, rhs, sm);
                    else if (N == 16) restrict_call<T, 16, 8>(L, Lc, into_old, blk, rhs, sm);
                    else restrict_call<T, 8, 8>(L, Lc, into_old, blk, rhs, sm))
        if (into_old) OCTMG_PHASE(Lc.nblocks, copy_parents_body3(NC, Lc, blk, rhs))
        // the coarse level's refinement ghosts come from level il-2; level 0
        // has none (it is complete), so Lcc is only read when il >= 2
        OCTMG_PHASE(Lc.nblocks, if (NC == 16) fas_rhs_call<T, 16>(Lc, Lcc, blk, rhs, sm);
                    else fas_rhs_call<T, 8>(Lc, Lcc, blk, rhs, sm))
    }
    OCTMG_PHASE(16, coarse_call<T>(P->L[0], P->M, P->S, blk, rhs, smem))
    for (int il = 1; il <= top; il++) {
        const LV<T> &L = P->L[il], &Lc = P->L[il - 1];
        const int N = P->N[il], NC = P->N[il - 1];
        OCTMG_PHASE(L.nblocks, if (N == 16 && NC == 16) prolong_call<T, 16, 16>(L, Lc, blk, rhs, sm);
                    else if (N == 16) prolong_call<T, 16, 8>(L, Lc, blk, rhs, sm);
                    else prolong_call<T, 8, 8>(L, Lc, blk, rhs, sm))
        for (int st = 0; st < P->n_up; st++)
            for (int color = 0; color < 2; color++)
                OCTMG_PHASE(L.nblocks, if (N == 16) gs_call<T, 16>(L, Lc, color, blk, rhs, sm);
                            else gs_call<T, 8>(L, Lc, color, blk, rhs, sm))
    }
#undef OCTMG_PHASE
}

// threads per colour of the colour-pair FAS right-hand side: 512 on 16^3
// blocks when the launch has at most one workgroup per CU (measured 0.1-0.3
// us faster per launch on the levels of 1-64 blocks at 256^3), else 256
// (two workgroups then share a CU: 20.9 us against 22.9 us on 512 blocks;
// restriction and residual measured slower with 512 at the finest level)
constexpr long long kWideFasMax = 256;

int grid_for(long long n) {
    long long g = (n + 255) / 256;
    return (int)(g < 4096 ? (g < 1 ? 1 : g) : 4096);
}

}  // namespace

// --------------------------------------------------------------- dispatch
// launches with more workgroups than this load g after the stencil in the
// residual and the restriction (two workgroups per CU on 256 CUs)
constexpr long long kLateMin = 512;

#define OCTMG_DN(D_, N_, CALL) \
    if (D == D_ && N == N_) { CALL; return hipGetLastError(); }

template <typename T>
hipError_t launch_gs_half(int D, int N, const LV<T> &L, const LV<T> &Lc, int color, int nrhs, hipStream_t s) {
    if (L.nblocks == 0) return hipSuccess;
    dim3 grid(L.nblocks, nrhs);
#define GS(D_, N_) OCTMG_DN(D_, N_, hipLaunchKernelGGL((k_gs_half<T, D_, N_>), grid, dim3(Blk<D_, N_>::THREADS), 0, s, L, Lc, color))
    // 16^3 blocks: launches of at most pair_max workgroups split a colour
    // over 512 threads (4 cells each instead of 8)
    if (D == 3 && N == 16 && (long long)L.nblocks * nrhs <= L.pair_max) {
        hipLaunchKernelGGL((k_gs_half3<T, 16, 512, cell_pairs<16>()>), grid, dim3(512), 0, s, L, Lc, color);
        return hipGetLastError();
    }
#define GS3(N_) OCTMG_DN(3, N_, hipLaunchKernelGGL((k_gs_half3<T, N_, 256, cell_pairs<N_>()>), grid, dim3(256), 0, s, L, Lc, color))
    GS3(16) GS3(8) GS(2, 8) GS(2, 16)
#undef GS3
#undef GS
    return hipErrorInvalidValue;
}

hipError_t launch_gs_half_update(int N, const LV<float> &L, const LV<float> &Lc, const LV<double> &U, int keep,
                                 int nrhs, hipStream_t s) {
    if (L.nblocks == 0) return hipSuccess;
    dim3 grid(L.nblocks, nrhs);
    if (N == 16 && (long long)L.nblocks * nrhs <= L.pair_max)
        hipLaunchKernelGGL((k_gs_half3_update<16, 512, cell_pairs<16>()>), grid, dim3(512), 0, s, L, Lc, U, keep);
    else if (N == 16)
        hipLaunchKernelGGL((k_gs_half3_update<16, 256, cell_pairs<16>()>), grid, dim3(256), 0, s, L, Lc, U, keep);
    else if (N == 8)
        hipLaunchKernelGGL((k_gs_half3_update<8, 256, cell_pairs<8>()>), grid, dim3(256), 0, s, L, Lc, U, keep);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

#define OCTMG_DNC(D_, N_, NC_, CALL) \
    if (D == D_ && N == N_ && Nc == NC_) { CALL; return hipGetLastError(); }

template <typename T>
hipError_t launch_restrict_fas(int D, int N, int Nc, const LV<T> &L, const LV<T> &Lc, int into_old, int nrhs,
                               hipStream_t s) {
    if (L.nblocks == 0) return hipSuccess;
    dim3 grid(L.nblocks, nrhs);
#define RF(D_, N_, NC_) OCTMG_DNC(D_, N_, NC_, hipLaunchKernelGGL((k_restrict_fas<T, D_, N_, NC_>), grid, dim3(256), 0, s, L, Lc, into_old))
    const bool pair = (long long)L.nblocks * nrhs <= L.pair_max;
    const bool late = (long long)L.nblocks * nrhs > kLateMin;
#define RF3(N_, NC_)                                                                                              \
    OCTMG_DNC(3, N_, NC_,                                                                                         \
              if (pair && late) hipLaunchKernelGGL((k_restrict_fas3_pair<T, N_, NC_, 256, true>), grid, dim3(512), 0, s, L, Lc, into_old); \
              else if (pair) hipLaunchKernelGGL((k_restrict_fas3_pair<T, N_, NC_, 256, false>), grid, dim3(512), 0, s, L, Lc, into_old); \
              else hipLaunchKernelGGL((k_restrict_fas3<T, N_, NC_>), grid, dim3(256), 0, s, L, Lc, into_old))
    RF3(16, 16) RF3(16, 8) RF3(8, 8) RF(2, 8, 8) RF(2, 16, 16) RF(2, 16, 8)
#undef RF3
#undef RF
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_single_block(int Nc, const LV<T> &L, const LV<T> &Lc, int fas, int restrict_to, int steps, int into_old,
                               int nrhs, hipStream_t s) {
    if (L.nblocks != 1 || L.nb != 1 || L.n != 16 || steps < 0) return hipErrorInvalidValue;
    dim3 grid(1, nrhs);
    if (!restrict_to) {
        if (fas) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_single_block3<T, false, false, 8>), grid, dim3(1024), 0, s, L, Lc, steps, into_old);
        return hipGetLastError();
    }
#define SB(F_, NC_)                                                                                              \
    if (!!fas == F_ && Nc == NC_) {                                                                              \
        hipLaunchKernelGGL((k_single_block3<T, F_, true, NC_>), grid, dim3(1024), 0, s, L, Lc, steps, into_old); \
        return hipGetLastError();                                                                                \
    }
    SB(true, 8) SB(false, 8) SB(true, 16) SB(false, 16)
#undef SB
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_copy_parents(int D, int N, const LV<T> &L, int nrhs, hipStream_t s, int leaves_only) {
    if (L.nblocks == 0) return hipSuccess;
    dim3 grid(L.nblocks, nrhs);
#define CP(D_, N_) OCTMG_DN(D_, N_, hipLaunchKernelGGL((k_copy_parents<T, D_, N_>), grid, dim3(256), 0, s, L, leaves_only))
    CP(3, 16) CP(3, 8) CP(2, 8) CP(2, 16)
#undef CP
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_restrict_rhs(int D, int N, int Nc, const LV<T> &L, const LV<T> &Lc, int nrhs, hipStream_t s) {
    if (L.nblocks == 0) return hipSuccess;
    dim3 grid(L.nblocks, nrhs);
#define RR(D_, N_, NC_) OCTMG_DNC(D_, N_, NC_, hipLaunchKernelGGL((k_restrict_rhs<T, D_, N_, NC_>), grid, dim3(256), 0, s, L, Lc))
    RR(3, 16, 16) RR(3, 16, 8) RR(3, 8, 8) RR(2, 8, 8) RR(2, 16, 16) RR(2, 16, 8)
#undef RR
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_restrict_phi(int D, int N, int Nc, const LV<T> &L, const LV<T> &Lc, int nrhs, hipStream_t s) {
    if (L.nblocks == 0) return hipSuccess;
    dim3 grid(L.nblocks, nrhs);
#define RP(D_, N_, NC_) OCTMG_DNC(D_, N_, NC_, hipLaunchKernelGGL((k_restrict_phi<T, D_, N_, NC_>), grid, dim3(256), 0, s, L, Lc))
    RP(3, 16, 16) RP(3, 16, 8) RP(3, 8, 8) RP(2, 8, 8) RP(2, 16, 16) RP(2, 16, 8)
#undef RP
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_fas_rhs(int D, int N, const LV<T> &L, const LV<T> &Lc, int parents_only, int nrhs, hipStream_t s) {
    if (L.nblocks == 0) return hipSuccess;
    dim3 grid(L.nblocks, nrhs);
#define FR(D_, N_) OCTMG_DN(D_, N_, hipLaunchKernelGGL((k_fas_rhs<T, D_, N_>), grid, dim3(Blk<D_, N_>::THREADS), 0, s, L, Lc, parents_only))
    const bool pair = (long long)L.nblocks * nrhs <= L.pair_max;
    const bool wide = (long long)L.nblocks * nrhs <= kWideFasMax;
    if (D == 3 && N == 16 && pair && wide) {
        hipLaunchKernelGGL((k_fas_rhs3_pair<T, 16, 512>), grid, dim3(1024), 0, s, L, Lc, parents_only);
        return hipGetLastError();
    }
#define FR3(N_)                                                                                                 \
    OCTMG_DN(3, N_, if (pair) hipLaunchKernelGGL((k_fas_rhs3_pair<T, N_, 256>), grid, dim3(512), 0, s, L, Lc, parents_only); \
             else hipLaunchKernelGGL((k_fas_rhs3<T, N_>), grid, dim3(256), 0, s, L, Lc, parents_only))
    FR3(16) FR3(8) FR(2, 8) FR(2, 16)
#undef FR3
#undef FR
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_fas_gs(int D, int N, const LV<T> &L, const LV<T> &Lc, int own_to_phi, int nrhs, hipStream_t s) {
    if (L.nblocks == 0) return hipSuccess;
    dim3 grid(L.nblocks, nrhs);
    if (D == 3 && N == 16 && (long long)L.nblocks * nrhs <= kWideFasMax) {
        hipLaunchKernelGGL((k_fas_gs3_pair<T, 16, 512>), grid, dim3(1024), 0, s, L, Lc, own_to_phi);
        return hipGetLastError();
    }
#define FG3(N_) OCTMG_DN(3, N_, hipLaunchKernelGGL((k_fas_gs3_pair<T, N_, 256>), grid, dim3(512), 0, s, L, Lc, own_to_phi))
    FG3(16) FG3(8)
#undef FG3
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_prolong(int D, int N, int Nc, const LV<T> &L, const LV<T> &Lc, int solution_mode, int nrhs,
                          hipStream_t s) {
    if (L.nblocks == 0) return hipSuccess;
    dim3 grid(L.nblocks, nrhs);
#define PR(D_, N_, NC_) OCTMG_DNC(D_, N_, NC_, hipLaunchKernelGGL((k_prolong<T, D_, N_, NC_>), grid, dim3(256), 0, s, L, Lc, solution_mode))
    const bool wide = (long long)L.nblocks * nrhs <= L.pair_max;
#define PR3(N_, NC_)                                                                                            \
    OCTMG_DNC(3, N_, NC_,                                                                                       \
              if (solution_mode) {                                                                              \
                  if (wide) hipLaunchKernelGGL((k_prolong3<T, N_, NC_, true, 512>), grid, dim3(512), 0, s, L, Lc); \
                  else hipLaunchKernelGGL((k_prolong3<T, N_, NC_, true, 256>), grid, dim3(256), 0, s, L, Lc);    \
              } else {                                                                                          \
                  if (wide) hipLaunchKernelGGL((k_prolong3<T, N_, NC_, false, 512>), grid, dim3(512), 0, s, L, Lc); \
                  else hipLaunchKernelGGL((k_prolong3<T, N_, NC_, false, 256>), grid, dim3(256), 0, s, L, Lc);   \
              })
    PR3(16, 16) PR3(16, 8) PR3(8, 8) PR(2, 8, 8) PR(2, 16, 16) PR(2, 16, 8)
#undef PR3
#undef PR
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_prolong_gs(int N, int Nc, const LV<T> &L, const LV<T> &Lc, int nrhs, hipStream_t s) {
    if (L.nblocks == 0) return hipSuccess;
    if (!L.own) return hipErrorInvalidValue;
    dim3 grid(L.nblocks, nrhs);
    const bool wide = N == 16 && (long long)L.nblocks * nrhs <= L.pair_max;
    if (N == 16 && Nc == 16) {
        if (wide) hipLaunchKernelGGL((k_prolong_gs3<T, 16, 16, 512, cell_pairs<16>()>), grid, dim3(512), 0, s, L, Lc);
        else hipLaunchKernelGGL((k_prolong_gs3<T, 16, 16, 256, cell_pairs<16>()>), grid, dim3(256), 0, s, L, Lc);
    } else if (N == 16 && Nc == 8) {
        if (wide) hipLaunchKernelGGL((k_prolong_gs3<T, 16, 8, 512, cell_pairs<16>()>), grid, dim3(512), 0, s, L, Lc);
        else hipLaunchKernelGGL((k_prolong_gs3<T, 16, 8, 256, cell_pairs<16>()>), grid, dim3(256), 0, s, L, Lc);
    } else if (N == 8 && Nc == 8) {
        hipLaunchKernelGGL((k_prolong_gs3<T, 8, 8, 256, false>), grid, dim3(256), 0, s, L, Lc);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_solve(int D, const LV<T> &L0, const double *M, const double *S, int fas, int nrhs,
                               hipStream_t s) {
    if (D == 3) {
        if (fas) hipLaunchKernelGGL((k_coarse_solve<T, 3, true>), dim3(512 / 8, nrhs), dim3(256), 0, s, L0, M, S);
        else hipLaunchKernelGGL((k_coarse_solve<T, 3, false>), dim3(512 / 8, nrhs), dim3(256), 0, s, L0, M, S);
    } else {
        if (fas) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_coarse_solve<T, 2, false>), dim3(64 / 16, nrhs), dim3(256), 0, s, L0, M, S);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_residual_max(int D, int N, const LV<T> &L, const LV<T> &Lc, int phi_zero, unsigned long long *out,
                               int nrhs, hipStream_t s) {
    if (L.nblocks == 0) return hipSuccess;
    dim3 grid(L.nblocks, nrhs);
    const bool pair = (long long)L.nblocks * nrhs <= L.pair_max;
    const bool late = (long long)L.nblocks * nrhs > kLateMin;
#define RM(D_, N_)                                                                                                  \
    if (D == D_ && N == N_) {                                                                                       \
        if (phi_zero) hipLaunchKernelGGL((k_residual_max<T, D_, N_, true>), grid, dim3(Blk<D_, N_>::THREADS), 0, s, L, Lc, out); \
        else hipLaunchKernelGGL((k_residual_max<T, D_, N_, false>), grid, dim3(Blk<D_, N_>::THREADS), 0, s, L, Lc, out); \
        return hipGetLastError();                                                                                   \
    }
#define RM3(N_)                                                                                                     \
    if (D == 3 && N == N_) {                                                                                        \
        if (phi_zero) hipLaunchKernelGGL((k_residual_max3<T, N_, true>), grid, dim3(256), 0, s, L, Lc, out);            \
        else if (pair && late) hipLaunchKernelGGL((k_residual_max3_pair<T, N_, 256, true>), grid, dim3(512), 0, s, L, Lc, out); \
        else if (pair) hipLaunchKernelGGL((k_residual_max3_pair<T, N_, 256, false>), grid, dim3(512), 0, s, L, Lc, out); \
        else hipLaunchKernelGGL((k_residual_max3<T, N_, false>), grid, dim3(256), 0, s, L, Lc, out);                    \
        return hipGetLastError();                                                                                   \
    }
    RM3(16) RM3(8) RM(2, 8) RM(2, 16)
#undef RM3
#undef RM
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_small_vcycle(const SmallLevels<T> *P, int top, int grid, hipStream_t s) {
    const SmallLevels<T> *arg = P;
    int top_arg = top;
    void *args[] = {&arg, &top_arg};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_small_vcycle<T>), dim3(grid), dim3(256), args,
                                      0, s);
}

template <typename T>
hipError_t small_vcycle_max_grid(int *grid) {
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&k_small_vcycle<T>), 256, 0);
    if (e != hipSuccess) return e;
    *grid = per_cu * prop.multiProcessorCount;
    return hipSuccess;
}
template hipError_t launch_small_vcycle<double>(const SmallLevels<double> *, int, int, hipStream_t);
template hipError_t launch_small_vcycle<float>(const SmallLevels<float> *, int, int, hipStream_t);
template hipError_t small_vcycle_max_grid<double>(int *);
template hipError_t small_vcycle_max_grid<float>(int *);

hipError_t launch_scatter_leaf(int D, int N, const LV<double> &L, const int *lb, int nlb, const double *src,
                               long long src_stride, long long base, int field, int nrhs, hipStream_t s) {
    if (nlb == 0) return hipSuccess;
    dim3 grid(nlb, nrhs);
#define SC(D_, N_) OCTMG_DN(D_, N_, hipLaunchKernelGGL((k_scatter_leaf<D_, N_>), grid, dim3(256), 0, s, L, lb, src, src_stride, base, field))
    SC(3, 16) SC(3, 8) SC(2, 8) SC(2, 16)
#undef SC
    return hipErrorInvalidValue;
}

hipError_t launch_gather_leaf(int D, int N, const LV<double> &L, const int *lb, int nlb, double *dst,
                              long long dst_stride, long long base, int nrhs, hipStream_t s) {
    if (nlb == 0) return hipSuccess;
    dim3 grid(nlb, nrhs);
#define GA(D_, N_) OCTMG_DN(D_, N_, hipLaunchKernelGGL((k_gather_leaf<D_, N_>), grid, dim3(256), 0, s, L, lb, dst, dst_stride, base))
    GA(3, 16) GA(3, 8) GA(2, 8) GA(2, 16)
#undef GA
    return hipErrorInvalidValue;
}

hipError_t launch_gradient(int D, int N, const LV<double> &L, const LV<double> &Lc, const int *lb, int nlb,
                           const int *meta, const double *d6, const int *inside, const double *pb, int inside_zero,
                           double *out, long long out_stride, long long base, int nrhs, hipStream_t s) {
    if (nlb == 0) return hipSuccess;
    dim3 grid(nlb, nrhs);
#define GR(D_, N_) OCTMG_DN(D_, N_, hipLaunchKernelGGL((k_gradient<D_, N_>), grid, dim3(256), 0, s, L, Lc, lb, meta, d6, inside, pb, inside_zero, out, out_stride, base))
    GR(3, 16) GR(3, 8) GR(2, 8) GR(2, 16)
#undef GR
    return hipErrorInvalidValue;
}

hipError_t launch_remap(int D, int N, const LV<double> &Ln, int il, const LV<double> *Lold, const int *nb_old,
                        const int *lb, int nlb, int nrhs, hipStream_t s) {
    if (nlb == 0) return hipSuccess;
    dim3 grid(nlb, nrhs);
#define RM(D_, N_) OCTMG_DN(D_, N_, hipLaunchKernelGGL((k_remap<D_, N_>), grid, dim3(256), 0, s, Ln, il, Lold, nb_old, lb))
    RM(3, 16) RM(3, 8) RM(2, 8) RM(2, 16)
#undef RM
    return hipErrorInvalidValue;
}

hipError_t launch_level_copy(int D, int N, double *split, double *canon, int nblocks, int to_split, hipStream_t s) {
    if (nblocks == 0) return hipSuccess;
#define LC(D_, N_) OCTMG_DN(D_, N_, hipLaunchKernelGGL((k_level_copy<D_, N_>), dim3(nblocks), dim3(256), 0, s, split, canon, to_split))
    LC(3, 16) LC(3, 8) LC(2, 8) LC(2, 16)
#undef LC
    return hipErrorInvalidValue;
}

hipError_t launch_defect(int D, int N, const LV<double> &L, const LV<double> &Lc, LV<float> L32, const int *lb,
                         int nlb, unsigned long long *out, int nrhs, hipStream_t s, int red_preset) {
    if (nlb == 0) return hipSuccess;
    dim3 grid(nlb, nrhs);
#define DF(D_, N_) OCTMG_DN(D_, N_, hipLaunchKernelGGL((k_defect<D_, N_>), grid, dim3(Blk<D_, N_>::THREADS), 0, s, L, Lc, L32, lb, out))
    const bool pair = (long long)nlb * nrhs <= L.pair_max, late = (long long)nlb * nrhs > kLateMin;
#define DF3(N_)                                                                                                    \
    OCTMG_DN(3, N_,                                                                                                \
             if (pair && late) hipLaunchKernelGGL((k_defect3_pair<N_, 256, true>), grid, dim3(512), 0, s, L, Lc, L32, lb, out, red_preset); \
             else if (pair) hipLaunchKernelGGL((k_defect3_pair<N_, 256, false>), grid, dim3(512), 0, s, L, Lc, L32, lb, out, red_preset); \
             else hipLaunchKernelGGL((k_defect3<N_>), grid, dim3(256), 0, s, L, Lc, L32, lb, out, red_preset))
    DF3(16) DF3(8) DF(2, 8) DF(2, 16)
#undef DF3
#undef DF
    return hipErrorInvalidValue;
}

hipError_t launch_update(int D, int N, const LV<double> &L, LV<float> L32, const int *lb, int nlb, int nrhs,
                         hipStream_t s) {
    if (nlb == 0) return hipSuccess;
    dim3 grid(nlb, nrhs);
#define UP(D_, N_) OCTMG_DN(D_, N_, hipLaunchKernelGGL((k_update<D_, N_>), grid, dim3(256), 0, s, L, L32, lb))
    UP(3, 16) UP(3, 8) UP(2, 8) UP(2, 16)
#undef UP
    return hipErrorInvalidValue;
}

hipError_t launch_boundary_terms(int D, const int *meta, const double *cfull, int nrec, const double *vals,
                                 double *b64, float *b32, hipStream_t s) {
    if (nrec == 0) return hipSuccess;
    hipLaunchKernelGGL(k_boundary_terms, dim3((nrec + 255) / 256), dim3(256), 0, s, D, meta, cfull, nrec, vals, b64, b32);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, long long n, double v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fillf(float *p, long long n, float v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fillf, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, long long n, unsigned long long v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_norm_reduce(unsigned long long *slots, unsigned long long *norm, unsigned long long *mapped,
                              int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_norm_reduce, dim3(1), dim3(64), 0, s, slots, norm, mapped, nrhs);
    return hipGetLastError();
}
hipError_t launch_converge(const unsigned long long *norm, const double *thresh, int *active, double *hist, int c,
                           int nrhs, int *cbase, int max_cycles, int advance, hipStream_t s) {
    hipLaunchKernelGGL(k_converge, dim3(1), dim3(256), 0, s, norm, thresh, active, hist, c, nrhs, cbase, max_cycles,
                       advance);
    return hipGetLastError();
}
hipError_t launch_copy_d2f(const double *src, float *dst, long long n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_d2f, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}
hipError_t launch_copy_f2d(const float *src, double *dst, long long n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_f2d, dim3(grid_for(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}
hipError_t launch_check_finite(const double *p, long long n, int *flag, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n)), dim3(256), 0, s, p, n, flag);
    return hipGetLastError();
}

#define OCTMG_INST(T)                                                                                              \
    template hipError_t launch_gs_half<T>(int, int, const LV<T> &, const LV<T> &, int, int, hipStream_t);           \
    template hipError_t launch_restrict_fas<T>(int, int, int, const LV<T> &, const LV<T> &, int, int, hipStream_t); \
    template hipError_t launch_copy_parents<T>(int, int, const LV<T> &, int, hipStream_t, int);                    \
    template hipError_t launch_restrict_rhs<T>(int, int, int, const LV<T> &, const LV<T> &, int, hipStream_t);      \
    template hipError_t launch_restrict_phi<T>(int, int, int, const LV<T> &, const LV<T> &, int, hipStream_t);      \
    template hipError_t launch_fas_rhs<T>(int, int, const LV<T> &, const LV<T> &, int, int, hipStream_t);           \
    template hipError_t launch_fas_gs<T>(int, int, const LV<T> &, const LV<T> &, int, int, hipStream_t);             \
    template hipError_t launch_single_block<T>(int, const LV<T> &, const LV<T> &, int, int, int, int, int, hipStream_t); \
    template hipError_t launch_prolong<T>(int, int, int, const LV<T> &, const LV<T> &, int, int, hipStream_t);      \
    template hipError_t launch_prolong_gs<T>(int, int, const LV<T> &, const LV<T> &, int, hipStream_t);            \
    template hipError_t launch_coarse_solve<T>(int, const LV<T> &, const double *, const double *, int, int, hipStream_t); \
    template hipError_t launch_residual_max<T>(int, int, const LV<T> &, const LV<T> &, int, unsigned long long *, int, hipStream_t);
OCTMG_INST(double)
OCTMG_INST(float)

}  // namespace octmg
