// FP64 interface setup.
//
// For every cell of a level: the boundary mask of eq. (boundary-mask), the
// relative distances d of Sec. 3.2 (bisection when a link is bracketed,
// golden-section bracket search otherwise), the unresolved-boundary search
// of Sec. 3.6.3 on parent blocks of coarse levels, and the interface stencil
// of eqs. (lpl-1d-lsf)/(lpl-2d-lsf) with cut links moved to the right-hand
// side (Sec. 3.6.2).  The level-set decisions must not depend on rounding
// shortcuts, so this file is compiled with -ffp-contract=off and uses only
// + - * / sqrt and comparisons (all correctly rounded).
//
// The per-cell analysis is written once, for host and device: the built-in
// level sets run it in the setup kernels, a level set given as a host
// function runs it on the host (host_setup_count / host_setup_emit), with
// the same results for the same f.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include "lsf.hpp"
#include "octmg_internal.hpp"

namespace octmg {
namespace {

__host__ __device__ inline Lsf lsf_of(const SetupLevel &S) {
    return Lsf{S.lsf_kind, S.lsf_n, S.D, S.lsf_params, S.lsf_fn, S.lsf_user};
}

__host__ __device__ inline double centre(const SetupLevel &S, int a, int gi) {
    return S.lo[a] + ((double)gi + 0.5) * S.dx;
}

__host__ __device__ inline void along(const double *a, const double *b, double t, double *x) {
    for (int c = 0; c < 3; c++) x[c] = a[c] + t * (b[c] - a[c]);
}

// bisection on [0, thi] of a->b; sign test f(a) f(x) <= 0
template <class F>
__host__ __device__ double bisect(const SetupLevel &S, const F &f, const double *a, const double *b, double fa,
                                  double thi) {
    double lo = 0.0, hi = thi, x[3];
    for (int it = 0; it < S.nbisect; it++) {
        double mid = 0.5 * (lo + hi);
        along(a, b, mid, x);
        if (fa * f(x) <= 0.0) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// root of f on a->b (t in (0,1]); *hit = 0 when no bracket is found within
// the golden-section evaluation budget
template <class F>
__host__ __device__ double root_on_link(const SetupLevel &S, const F &f, const double *a, const double *b, double fa,
                                        int *hit) {
    double x[3];
    *hit = 1;
    if (fa * f(b) <= 0.0) return bisect(S, f, a, b, fa, 1.0);
    const double rho = 0.5 * (sqrt_rn(5.0) - 1.0);
    double lo = 0.0, hi = 1.0;
    double t1 = hi - rho * (hi - lo), t2 = lo + rho * (hi - lo);
    along(a, b, t1, x);
    double h1 = fa * f(x);
    if (h1 <= 0.0) return bisect(S, f, a, b, fa, t1);
    along(a, b, t2, x);
    double h2 = fa * f(x);
    if (h2 <= 0.0) return bisect(S, f, a, b, fa, t2);
    for (int used = 2; used < S.ngolden; used++) {
        if (h1 < h2) {
            hi = t2;
            t2 = t1;
            h2 = h1;
            t1 = hi - rho * (hi - lo);
            along(a, b, t1, x);
            h1 = fa * f(x);
            if (h1 <= 0.0) return bisect(S, f, a, b, fa, t1);
        } else {
            lo = t1;
            t1 = t2;
            h1 = h2;
            t2 = lo + rho * (hi - lo);
            along(a, b, t2, x);
            h2 = fa * f(x);
            if (h2 <= 0.0) return bisect(S, f, a, b, fa, t2);
        }
    }
    *hit = 0;
    return 1.0;
}

// Sec. 3.6.3: descent with step w_min towards f = 0, then a line search a->x.
template <class F>
__host__ __device__ int unresolved_search(const SetupLevel &S, const F &f, const double *a, double fa, double *dout,
                                          int *dir, double *x0) {
    const double w = S.w_min;
    double x[3] = {a[0], a[1], a[2]};
    const double sgn = fa > 0.0 ? 1.0 : -1.0;
    const int steps = (int)floor(S.dx / w);
    int hit = 0;
    for (int st = 0; st < steps; st++) {
        double gr[3] = {0.0, 0.0, 0.0}, n2 = 0.0;
        for (int c = 0; c < S.D; c++) {
            double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
            xp[c] = x[c] + w;
            xm[c] = x[c] - w;
            gr[c] = (f(xp) - f(xm)) / (2.0 * w);
            n2 = n2 + gr[c] * gr[c];
        }
        double nrm = sqrt_rn(n2);
        if (!(nrm > 0.0)) break;
        bool leaves = false;
        for (int c = 0; c < S.D; c++) {
            double step = -sgn * gr[c] / nrm;
            x[c] = x[c] + w * step;
            if (x[c] < S.lo[c] || x[c] > S.lo[c] + 1.0) leaves = true;
        }
        if (leaves) break;
        if (fa * f(x) <= 0.0) {
            hit = 1;
            break;
        }
    }
    if (!hit) return 0;
    double t = bisect(S, f, a, x, fa, 1.0), p[3], s2 = 0.0;
    along(a, x, t, p);
    for (int c = 0; c < S.D; c++) s2 = s2 + (p[c] - a[c]) * (p[c] - a[c]);
    double d = sqrt_rn(s2) / S.dx;
    if (!(d < 1.0)) return 0;
    double best = -1.0;
    int k = 0;
    for (int c = 0; c < S.D; c++) {
        double v = x[c] - a[c];
        if (v > best) { best = v; k = 2 * c + 1; }
        if (-v > best) { best = -v; k = 2 * c; }
    }
    *dout = d;
    *dir = k;
    for (int c = 0; c < 3; c++) x0[c] = p[c];
    return 1;
}

struct CellSetup {
    int cut, inside;
    double d[6];
    double x0[6][3];
};

// returns 1 if the cell carries a custom stencil (at least one cut link)
template <class F>
__host__ __device__ int analyse_cell(const SetupLevel &S, const F &f, int blk, int li, CellSetup &R) {
    const int4 p = S.pos[blk];
    int l[3] = {li % S.Nb, (li / S.Nb) % S.Nb, S.D == 3 ? li / (S.Nb * S.Nb) : 0};
    int g[3] = {p.x * S.Nb + l[0], p.y * S.Nb + l[1], S.D == 3 ? p.z * S.Nb + l[2] : 0};
    double a[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < S.D; c++) a[c] = centre(S, c, g[c]);
    const double fa = f(a);
    double n2 = 0.0;
    for (int c = 0; c < S.D; c++) {
        double xp[3] = {a[0], a[1], a[2]}, xm[3] = {a[0], a[1], a[2]};
        xp[c] = centre(S, c, g[c] + 1);
        xm[c] = centre(S, c, g[c] - 1);
        double gc = (f(xp) - f(xm)) / (2.0 * S.dx);
        n2 = n2 + gc * gc;
    }
    R.cut = 0;
    R.inside = fa < 0.0;
    for (int k = 0; k < 6; k++) R.d[k] = 1.0;
    if (!(fabs(fa) < S.mask_L * sqrt_rn(n2))) return 0;
    for (int k = 0; k < 2 * S.D; k++) {
        const int ax = k >> 1, s = (k & 1) ? 1 : -1;
        if (g[ax] + s < 0 || g[ax] + s >= S.n) continue;  // links leaving the domain
        double b[3] = {a[0], a[1], a[2]};
        b[ax] = centre(S, ax, g[ax] + s);
        int hit;
        double t = root_on_link(S, f, a, b, fa, &hit);
        if (hit) {
            R.d[k] = t;
            R.cut |= 1 << k;
            along(a, b, t, R.x0[k]);
        }
    }
    if (!R.cut && !S.leaf[blk] && S.w_min > 0.0 && S.dx > S.w_min) {
        double d, x0[3];
        int k;
        if (unresolved_search(S, f, a, fa, &d, &k, x0)) {
            R.d[k] = d;
            R.cut = 1 << k;
            for (int c = 0; c < 3; c++) R.x0[k][c] = x0[c];
        }
    }
    return R.cut != 0;
}

__host__ __device__ inline int split_index(int D, int N, int li) {
    const int i = li % N, j = (li / N) % N, k = D == 3 ? li / (N * N) : 0;
    const int half = (D == 3 ? N * N * N : N * N) / 2;
    return ((i + j + k) & 1) * half + (k * N + j) * (N / 2) + (i >> 1);
}

// Output arrays of the record pass (device or host memory).
struct EmitOut {
    const int *map_off;
    int *map, *meta;
    double *d6, *cfull, *rec8;
    float *rec8f;
    double *pts;
    int *inside;
};

// The stencil of eqs. (lpl-1d-lsf)/(lpl-2d-lsf) of one analysed cell as
// record r with its cut-link points from slot q on; returns the next slot.
__host__ __device__ int emit_cell(const SetupLevel &S, const CellSetup &R, int blk, int li, int r, int q,
                                  const EmitOut &o) {
    const double dx2 = S.dx * S.dx;
    double c[6] = {0, 0, 0, 0, 0, 0}, diag = 0.0;
    for (int ax = 0; ax < S.D; ax++) {
        double dm = R.d[2 * ax], dp = R.d[2 * ax + 1];
        c[2 * ax] = 2.0 / ((dm + dp) * dm * dx2);
        c[2 * ax + 1] = 2.0 / ((dm + dp) * dp * dx2);
        diag = diag - c[2 * ax] - c[2 * ax + 1];
    }
    const int si = split_index(S.D, S.Nb, li);
    o.meta[4 * r + 0] = blk;
    o.meta[4 * r + 1] = si;
    o.meta[4 * r + 2] = R.cut;
    o.meta[4 * r + 3] = q;
    o.inside[r] = R.inside;
    for (int k = 0; k < 6; k++) {
        o.d6[6 * r + k] = R.d[k];
        o.cfull[6 * r + k] = c[k];
        double hot = (R.cut >> k & 1) ? 0.0 : c[k];
        o.rec8[8 * r + k] = hot;
        o.rec8f[8 * r + k] = (float)hot;
    }
    o.rec8[8 * r + 6] = diag;
    o.rec8[8 * r + 7] = 1.0 / diag;
    o.rec8f[8 * r + 6] = (float)diag;
    o.rec8f[8 * r + 7] = (float)(1.0 / diag);
    o.map[o.map_off[blk] + si] = r;
    for (int k = 0; k < 2 * S.D; k++) {
        if (!(R.cut >> k & 1)) continue;
        for (int cc = 0; cc < 3; cc++) o.pts[3 * q + cc] = R.x0[k][cc];
        q++;
    }
    return q;
}

constexpr int kSetupThreads = 256;

// The cells of a block are analysed by `split` workgroups, each taking one
// contiguous range of them, so that levels with few blocks still occupy the
// GPU (cell ranges never cross blocks: split divides the cells per block).
__global__ __launch_bounds__(kSetupThreads) void k_setup_count(SetupLevel S, int split, int *counts,
                                                                unsigned char *flags) {
    const int bi = (int)blockIdx.x / split, part = (int)blockIdx.x % split;
    const int blk = S.blocks ? S.blocks[bi] : bi;
    const int cpb = S.D == 3 ? S.Nb * S.Nb * S.Nb : S.Nb * S.Nb;
    const int span = cpb / split, c0 = part * span;
    unsigned char *fb = flags + (long long)blk * cpb;
    const Lsf f = lsf_of(S);
    int nrec = 0, npt = 0;
    CellSetup R;
    for (int li = c0 + (int)threadIdx.x; li < c0 + span; li += blockDim.x) {
        unsigned char fl = 0;
        if (analyse_cell(S, f, blk, li, R)) {
            const int pc = __builtin_popcount(R.cut);
            nrec++;
            npt += pc;
            fl = (unsigned char)(0x80 | pc);
        }
        fb[li] = fl;
    }
    __shared__ int sr[kSetupThreads], sp[kSetupThreads];
    sr[threadIdx.x] = nrec;
    sp[threadIdx.x] = npt;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            sp[threadIdx.x] += sp[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&counts[2 * blk], sr[0]);
        atomicAdd(&counts[2 * blk + 1], sp[0]);
    }
}

// Records of a block in canonical (x-fastest) cell order.  Within its cell
// range a workgroup gives thread t the contiguous cells
// [t*chunk, (t+1)*chunk); the flags of pass 1 give every thread its first
// record and point slot (the records and points of the block's cells before
// the range, plus an exclusive scan over the threads), and only the flagged
// cells are analysed again.
__global__ __launch_bounds__(kSetupThreads) void k_setup_emit(SetupLevel S, int split, const unsigned char *flags,
                                                               const int *rec_off, const int *pt_off, EmitOut o) {
    const int bi = (int)blockIdx.x / split, part = (int)blockIdx.x % split;
    const int blk = S.blocks ? S.blocks[bi] : bi;
    const int cpb = S.D == 3 ? S.Nb * S.Nb * S.Nb : S.Nb * S.Nb;
    const int span = cpb / split, c0 = part * span;
    const unsigned char *fb = flags + (long long)blk * cpb;
    const int chunk = (span + blockDim.x - 1) / blockDim.x;
    const int a0 = min(c0 + span, c0 + (int)threadIdx.x * chunk), a1 = min(c0 + span, a0 + chunk);
    int before_r = 0, before_p = 0;  // this thread's share of the cells before the range
    for (int li = threadIdx.x; li < c0; li += blockDim.x)
        if (fb[li]) {
            before_r++;
            before_p += fb[li] & 0x7f;
        }
    int nrec = 0, npt = 0;
    for (int li = a0; li < a1; li++)
        if (fb[li]) {
            nrec++;
            npt += fb[li] & 0x7f;
        }
    __shared__ int sr[kSetupThreads], sp[kSetupThreads], br[kSetupThreads], bp[kSetupThreads];
    sr[threadIdx.x] = nrec;
    sp[threadIdx.x] = npt;
    br[threadIdx.x] = before_r;
    bp[threadIdx.x] = before_p;
    __syncthreads();
    if (threadIdx.x == 0) {  // exclusive scan of the chunks, total before the range (setup only)
        int a = 0, b = 0, c = 0, d = 0;
        for (int t = 0; t < (int)blockDim.x; t++) {
            const int x = sr[t], y = sp[t];
            sr[t] = a;
            sp[t] = b;
            a += x;
            b += y;
            c += br[t];
            d += bp[t];
        }
        br[0] = c;
        bp[0] = d;
    }
    __syncthreads();
    int r = rec_off[blk] + br[0] + sr[threadIdx.x];
    int q = pt_off[blk] + bp[0] + sp[threadIdx.x];
    const Lsf f = lsf_of(S);
    CellSetup R;
    for (int li = a0; li < a1; li++) {
        if (!fb[li]) continue;
        analyse_cell(S, f, blk, li, R);
        q = emit_cell(S, R, blk, li, r, q, o);
        r++;
    }
}

// Records of a block that an adapted tree keeps unchanged (same level,
// position and leaf status): copied from the previous geometry with their
// block, record and point indices moved to the new offsets.
__global__ void k_reuse_records(const ReuseBlock *list, int cpb, ReuseArrays o, ReuseArrays n) {
    const ReuseBlock R = list[blockIdx.x];
    for (int t = threadIdx.x; t < R.nrec; t += blockDim.x) {
        const long ro = R.old_roff + t, rn = R.new_roff + t;
        n.meta[4 * rn + 0] = R.new_blk;
        n.meta[4 * rn + 1] = o.meta[4 * ro + 1];
        n.meta[4 * rn + 2] = o.meta[4 * ro + 2];
        n.meta[4 * rn + 3] = o.meta[4 * ro + 3] - R.old_poff + R.new_poff;
        for (int k = 0; k < 6; k++) {
            n.d6[6 * rn + k] = o.d6[6 * ro + k];
            n.cfull[6 * rn + k] = o.cfull[6 * ro + k];
        }
        for (int k = 0; k < 8; k++) {
            n.rec8[8 * rn + k] = o.rec8[8 * ro + k];
            n.rec8f[8 * rn + k] = o.rec8f[8 * ro + k];
        }
        n.inside[rn] = o.inside[ro];
    }
    for (int t = threadIdx.x; t < 3 * R.npt; t += blockDim.x)
        n.pts[3L * R.new_poff + t] = o.pts[3L * R.old_poff + t];
    if (R.new_moff >= 0)
        for (int c = threadIdx.x; c < cpb; c += blockDim.x) {
            const int v = o.map[(long)R.old_moff + c];
            n.map[(long)R.new_moff + c] = v >= 0 ? v - R.old_roff + R.new_roff : -1;
        }
}

// Dense operator of the single-block coarsest grid (canonical cell order),
// domain ghosts 2 phi_b - phi_in folded into the diagonal.
__global__ void k_coarse_assemble(int D, int Nb, double dx, const int *map, const double *rec8, int neumann,
                                  double *A) {
    const int n = D == 3 ? Nb * Nb * Nb : Nb * Nb;
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n) return;
    const double inv = 1.0 / (dx * dx);
    const int i = row % Nb, j = (row / Nb) % Nb, k = D == 3 ? row / (Nb * Nb) : 0;
    const int ri = map ? map[split_index(D, Nb, row)] : -1;
    for (int c = 0; c < n; c++) A[(long)row * n + c] = 0.0;
    double diag = ri >= 0 ? rec8[8 * ri + 6] : -2.0 * D * inv;
    for (int kk = 0; kk < 2 * D; kk++) {
        const int ax = kk >> 1, s = (kk & 1) ? 1 : -1;
        const double c = ri >= 0 ? rec8[8 * ri + kk] : inv;  // 0 for cut links
        if (c == 0.0) continue;
        int q[3] = {i, j, k};
        q[ax] += s;
        if (q[ax] < 0 || q[ax] >= Nb) {
            // ghost folded in: 2 phi_b - phi_i (Dirichlet), phi_i (zero flux)
            if ((neumann >> (2 * ax + (s > 0))) & 1) diag += c;
            else diag -= c;
            continue;
        }
        const int col = D == 3 ? (q[2] * Nb + q[1]) * Nb + q[0] : q[1] * Nb + q[0];
        A[(long)row * n + col] += c;
    }
    A[(long)row * n + row] += diag;
}

// Row-equilibrated Gauss-Jordan inverse with partial pivoting:
// S_i = 1 / max_j |A_ij|, M = (diag(S) A)^-1, A^-1 = M diag(S).  Step k runs
// as two launches: k_gj_pivot (one workgroup) picks the pivot row of column
// k (largest |A_rk|, r >= k, lowest r on ties), swaps it into row k, divides
// row k of A and M by the pivot and records the column multipliers;
// k_gj_eliminate (one thread per element) subtracts multiplier x row k from
// every other row.  Each element sees the same operations in the same order
// as in a one-workgroup elimination.
__global__ __launch_bounds__(256) void k_gj_scale(int n, double *A, double *M, double *S) {
    const int r = blockIdx.x;
    __shared__ double red[256];
    double m = 0.0;
    for (int c = threadIdx.x; c < n; c += blockDim.x) m = fmax(m, fabs(A[(long)r * n + c]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const double s = red[0] > 0.0 ? 1.0 / red[0] : 1.0;
    if (threadIdx.x == 0) S[r] = s;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        A[(long)r * n + c] *= s;
        M[(long)r * n + c] = r == c ? 1.0 : 0.0;
    }
}

__global__ __launch_bounds__(1024) void k_gj_pivot(int n, int k, double *A, double *M, double *mult, int *fail) {
    __shared__ double sval[1024];
    __shared__ int sidx[1024];
    if (*fail) return;
    const int t = threadIdx.x, T = blockDim.x;
    double best = -1.0;
    int bi = k;
    for (int r = k + t; r < n; r += T) {
        const double v = fabs(A[(long)r * n + k]);
        if (v > best) { best = v; bi = r; }
    }
    sval[t] = best;
    sidx[t] = bi;
    __syncthreads();
    for (int w = T / 2; w > 0; w >>= 1) {
        if (t < w && (sval[t + w] > sval[t] || (sval[t + w] == sval[t] && sidx[t + w] < sidx[t]))) {
            sval[t] = sval[t + w];
            sidx[t] = sidx[t + w];
        }
        __syncthreads();
    }
    const int p = sidx[0];
    if (!(sval[0] > 0.0)) {
        if (t == 0) *fail = 1;
        return;
    }
    if (p != k)
        for (int c = t; c < n; c += T) {
            const double x = A[(long)k * n + c], y = M[(long)k * n + c];
            A[(long)k * n + c] = A[(long)p * n + c];
            M[(long)k * n + c] = M[(long)p * n + c];
            A[(long)p * n + c] = x;
            M[(long)p * n + c] = y;
        }
    __syncthreads();
    const double inv = 1.0 / A[(long)k * n + k];
    __syncthreads();
    for (int c = t; c < n; c += T) {
        A[(long)k * n + c] *= inv;
        M[(long)k * n + c] *= inv;
    }
    __syncthreads();
    for (int r = t; r < n; r += T) mult[r] = r == k ? 0.0 : A[(long)r * n + k];
}

__global__ __launch_bounds__(256) void k_gj_eliminate(int n, int k, double *A, double *M, const double *mult,
                                                      const int *fail) {
    if (*fail) return;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * n) return;
    const int r = (int)(e / n), c = (int)(e % n);
    const double m = mult[r];
    if (m != 0.0) {
        A[e] -= m * A[(long)k * n + c];
        M[e] -= m * M[(long)k * n + c];
    }
}

}  // namespace

// workgroups per block: doubled while the launch has fewer than 32768
// workgroups and each keeps at least a cell per thread
static int setup_split(const SetupLevel &S, int nb) {
    const int cpb = S.D == 3 ? S.Nb * S.Nb * S.Nb : S.Nb * S.Nb;
    int split = 1;
    while (2 * split * kSetupThreads <= cpb && (long long)nb * split < 32768) split *= 2;
    return split;
}

hipError_t launch_setup_count(const SetupLevel &S, int *counts, unsigned char *flags, hipStream_t s) {
    if (S.nblocks == 0) return hipSuccess;
    const int nb = S.blocks ? S.nlist : S.nblocks;
    if (nb == 0) return hipSuccess;
    const int split = setup_split(S, nb);
    hipLaunchKernelGGL(k_setup_count, dim3(nb * split), dim3(kSetupThreads), 0, s, S, split, counts, flags);
    return hipGetLastError();
}

hipError_t launch_setup_emit(const SetupLevel &S, const unsigned char *flags, const int *rec_off, const int *pt_off,
                             const int *map_off, int *map, int *meta, double *d6, double *cfull, double *rec8,
                             float *rec8f, double *pts, int *inside, hipStream_t s) {
    if (S.nblocks == 0) return hipSuccess;
    const int nb = S.blocks ? S.nlist : S.nblocks;
    if (nb == 0) return hipSuccess;
    const int split = setup_split(S, nb);
    const EmitOut o{map_off, map, meta, d6, cfull, rec8, rec8f, pts, inside};
    hipLaunchKernelGGL(k_setup_emit, dim3(nb * split), dim3(kSetupThreads), 0, s, S, split, flags, rec_off, pt_off,
                       o);
    return hipGetLastError();
}

// Host passes for a level set given as a host function: the same cell
// analysis and records as k_setup_count / k_setup_emit, one cell after the
// other on the calling thread, into host arrays.
void host_setup_count(const SetupLevel &S, int *counts) {
    const int cpb = S.D == 3 ? S.Nb * S.Nb * S.Nb : S.Nb * S.Nb;
    const Lsf f = lsf_of(S);
    const int nb = S.blocks ? S.nlist : S.nblocks;
    CellSetup R;
    for (int i = 0; i < nb; i++) {
        const int blk = S.blocks ? S.blocks[i] : i;
        int nrec = 0, npt = 0;
        for (int li = 0; li < cpb; li++)
            if (analyse_cell(S, f, blk, li, R)) {
                nrec++;
                npt += __builtin_popcount(R.cut);
            }
        counts[2 * blk] = nrec;
        counts[2 * blk + 1] = npt;
    }
}

void host_setup_emit(const SetupLevel &S, const int *rec_off, const int *pt_off, const int *map_off, int *map,
                     int *meta, double *d6, double *cfull, double *rec8, float *rec8f, double *pts, int *inside) {
    const int cpb = S.D == 3 ? S.Nb * S.Nb * S.Nb : S.Nb * S.Nb;
    const Lsf f = lsf_of(S);
    const EmitOut o{map_off, map, meta, d6, cfull, rec8, rec8f, pts, inside};
    const int nb = S.blocks ? S.nlist : S.nblocks;
    CellSetup R;
    for (int i = 0; i < nb; i++) {
        const int blk = S.blocks ? S.blocks[i] : i;
        int r = rec_off[blk], q = pt_off[blk];
        for (int li = 0; li < cpb; li++) {
            if (!analyse_cell(S, f, blk, li, R)) continue;
            q = emit_cell(S, R, blk, li, r, q, o);
            r++;
        }
    }
}

hipError_t launch_reuse_records(const ReuseBlock *list, int nlist, int cpb, const ReuseArrays &o,
                                const ReuseArrays &n, hipStream_t s) {
    if (nlist == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reuse_records, dim3(nlist), dim3(256), 0, s, list, cpb, o, n);
    return hipGetLastError();
}

hipError_t launch_coarse_assemble(int D, int Nb, double dx, const int *map, const double *rec8, int neumann,
                                  double *A, hipStream_t s) {
    const int n = D == 3 ? Nb * Nb * Nb : Nb * Nb;
    hipLaunchKernelGGL(k_coarse_assemble, dim3((n + 127) / 128), dim3(128), 0, s, D, Nb, dx, map, rec8, neumann, A);
    return hipGetLastError();
}

hipError_t launch_gauss_jordan(int n, double *A, double *M, double *S, double *mult, int *fail, hipStream_t s) {
    if (n < 1 || n > 4096) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gj_scale, dim3(n), dim3(256), 0, s, n, A, M, S);
    const long ne = (long)n * n;
    for (int k = 0; k < n; k++) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, s, n, k, A, M, mult, fail);
        hipLaunchKernelGGL(k_gj_eliminate, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, n, k, A, M, mult,
                           (const int *)fail);
    }
    return hipGetLastError();
}

}  // namespace octmg
