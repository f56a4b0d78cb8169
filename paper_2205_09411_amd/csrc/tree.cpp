// Host construction of the block quadtree/octree (Sec. 2.1 of the paper):
// blocks of N^D cells, refinement halves the spacing and creates 2^D
// children, adjacent blocks differ by at most one level (2:1 balance over
// faces, edges and corners).  Below the root, single-block levels halve the
// cell count down to the directly solved coarse grid.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "lsf.hpp"
#include "octmg_internal.hpp"

namespace octmg {

double lsf_host(const octmg_geom_desc &d, const double *p, const double *x) {
    return Lsf{d.lsf_kind, d.lsf_n, d.dim, p, d.lsf_fn, d.lsf_user}(x);
}

namespace {

// dense occupancy of one tree level
struct Occ {
    int D, nb;
    std::vector<uint8_t> bits;
    long idx(int x, int y, int z) const { return D == 3 ? ((long)z * nb + y) * nb + x : (long)y * nb + x; }
    bool has(int x, int y, int z) const { return bits[idx(x, y, z)] != 0; }
};

uint64_t interleave(int D, int x, int y, int z) {
    uint64_t key = 0;
    for (int bit = 0; bit < 21; bit++) {
        key |= (uint64_t)((x >> bit) & 1) << (D * bit);
        key |= (uint64_t)((y >> bit) & 1) << (D * bit + 1);
        if (D == 3) key |= (uint64_t)((z >> bit) & 1) << (D * bit + 2);
    }
    return key;
}

void add_children(std::vector<Occ> &occ, int l, int x, int y, int z) {
    Occ &f = occ[l + 1];
    int nz = f.D == 3 ? 2 : 1;
    for (int c = 0; c < nz; c++)
        for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++) f.bits[f.idx(2 * x + a, 2 * y + b, f.D == 3 ? 2 * z + c : 0)] = 1;
}

}  // namespace

namespace {

bool check_desc(const octmg_geom_desc &d, std::string *err) {
    const int D = d.dim, N = d.block_n, lmax = d.max_level;
    if (D != 2 && D != 3) { *err = "dim must be 2 or 3"; return false; }
    if (N != 8 && N != 16) { *err = "block_n must be 8 or 16"; return false; }
    if (d.coarse_n != 8) { *err = "coarse_n must be 8"; return false; }
    if (lmax < 1 || lmax > 14) { *err = "max_level out of range"; return false; }
    if (d.lsf_kind == OCTMG_LSF_SPHERES && (d.lsf_n < 1 || !d.lsf_params)) { *err = "spheres need lsf_n >= 1 and params"; return false; }
    if (d.lsf_kind == OCTMG_LSF_CYLINDER_Z && !d.lsf_params) { *err = "cylinder needs params"; return false; }
    if (d.lsf_kind < OCTMG_LSF_NONE || d.lsf_kind > OCTMG_LSF_CALLBACK) { *err = "unknown lsf_kind"; return false; }
    if (d.lsf_kind == OCTMG_LSF_CALLBACK && !d.lsf_fn) { *err = "a callback level set needs lsf_fn"; return false; }
    if (d.lsf_kind == OCTMG_LSF_ELECTRODES && d.dim != 3) { *err = "the electrode level set is 3D"; return false; }
    if (d.refine_kind != OCTMG_REFINE_UNIFORM && d.refine_kind != OCTMG_REFINE_NEAR_INTERFACE) { *err = "unknown refine_kind"; return false; }
    if ((long)N << (lmax - 1) > (1L << 15)) { *err = "grid too large"; return false; }
    if (d.neumann_faces < 0 || d.neumann_faces >= (1 << (2 * D))) { *err = "neumann_faces has bits beyond the 2D faces"; return false; }
    if (d.uniform_level < 0 || d.uniform_level > lmax) { *err = "bad uniform_level"; return false; }

    return true;
}

std::vector<Occ> empty_occ(int D, int lmax) {
    std::vector<Occ> occ(lmax + 1);
    for (int l = 1; l <= lmax; l++) {
        occ[l].D = D;
        occ[l].nb = 1 << (l - 1);
        long cnt = 1;
        for (int a = 0; a < D; a++) cnt *= occ[l].nb;
        occ[l].bits.assign(cnt, 0);
    }
    return occ;
}

// 2:1 balance: a block at level l needs every neighbour region covered at
// level >= l-1, i.e. the level-(l-1) block containing each neighbour
// position must exist.  Missing ones are created by refining down from
// their deepest existing ancestor.  Processing fine to coarse handles the
// blocks this creates.
void balance(std::vector<Occ> &occ, int D, int lmax) {
    for (int l = lmax; l >= 3; l--) {
        const int nb = occ[l].nb, nz = D == 3 ? nb : 1;
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < nb; y++)
                for (int x = 0; x < nb; x++) {
                    if (!occ[l].has(x, y, z)) continue;
                    for (int oz = (D == 3 ? -1 : 0); oz <= (D == 3 ? 1 : 0); oz++)
                        for (int oy = -1; oy <= 1; oy++)
                            for (int ox = -1; ox <= 1; ox++) {
                                int qx = x + ox, qy = y + oy, qz = z + oz;
                                if (qx < 0 || qy < 0 || qz < 0 || qx >= nb || qy >= nb || qz >= nb) continue;
                                // required: block (l-1, q/2)
                                int tx = qx >> 1, ty = qy >> 1, tz = qz >> 1, tl = l - 1;
                                if (occ[tl].has(tx, ty, tz)) continue;
                                // deepest existing ancestor
                                int al = tl, ax = tx, ay = ty, az = tz;
                                while (!occ[al].has(ax, ay, az)) {
                                    al--;
                                    ax >>= 1;
                                    ay >>= 1;
                                    az >>= 1;
                                }
                                // refine along the chain down to level tl
                                while (al < tl) {
                                    add_children(occ, al, ax, ay, az);
                                    al++;
                                    int sh = tl - al;
                                    ax = tx >> sh;
                                    ay = ty >> sh;
                                    az = tz >> sh;
                                }
                            }
                }
    }

}

// levels (sub-root coarse levels first), Morton order, lookup tables, leaves
bool finalize(const octmg_geom_desc &d, const std::vector<Occ> &occ, Tree *out, std::string *err) {
    const int D = d.dim, N = d.block_n, lmax = d.max_level;
    Tree t;
    t.D = D;
    t.N = N;
    t.nsub = 0;
    for (int n = N; n > d.coarse_n; n >>= 1) t.nsub++;
    const int nlev = t.nsub + lmax;
    if (nlev > kMaxLevels) { *err = "too many levels"; return false; }
    t.lv.resize(nlev);
    for (int il = 0; il < nlev; il++) {
        TreeLevel &L = t.lv[il];
        const int l = il - t.nsub + 1;
        if (l <= 0) {
            L.n = N >> (1 - l);
            L.Nb = L.n;
            L.nb = 1;
        } else {
            L.n = N << (l - 1);
            L.Nb = N;
            L.nb = 1 << (l - 1);
        }
        const int nb = L.nb, nz = D == 3 ? nb : 1;
        std::vector<std::pair<uint64_t, std::array<int, 3>>> keyed;
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < nb; y++)
                for (int x = 0; x < nb; x++) {
                    if (l >= 1 && !occ[l].has(x, y, z)) continue;
                    keyed.push_back({interleave(D, x, y, z), {x, y, z}});
                }
        std::sort(keyed.begin(), keyed.end(),
                  [](const auto &a, const auto &b) { return a.first < b.first; });
        long cnt = 1;
        for (int a = 0; a < D; a++) cnt *= nb;
        L.lut.assign(cnt, -1);
        L.pos.resize(keyed.size() * 3);
        L.leaf.resize(keyed.size());
        for (size_t i = 0; i < keyed.size(); i++) {
            const auto &p = keyed[i].second;
            for (int a = 0; a < 3; a++) L.pos[3 * i + a] = p[a];
            L.lut[D == 3 ? ((long)p[2] * nb + p[1]) * nb + p[0] : (long)p[1] * nb + p[0]] = (int)i;
            bool leaf;
            if (l <= 0) leaf = false;
            else if (l == lmax) leaf = true;
            else leaf = !occ[l + 1].has(2 * p[0], 2 * p[1], D == 3 ? 2 * p[2] : 0);
            L.leaf[i] = leaf;
            if (leaf && l < lmax) t.adaptive = true;
        }
    }
    *out = std::move(t);
    return true;
}

}  // namespace

bool build_tree(const octmg_geom_desc &d, Tree *out, std::string *err) {
    if (!check_desc(d, err)) return false;
    const int D = d.dim, lmax = d.max_level;
    std::vector<Occ> occ = empty_occ(D, lmax);
    occ[1].bits[0] = 1;
    for (int l = 1; l < lmax; l++) {
        const int nb = occ[l].nb, nz = D == 3 ? nb : 1;
        const double w = 1.0 / (double)nb;
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < nb; y++)
                for (int x = 0; x < nb; x++) {
                    if (!occ[l].has(x, y, z)) continue;
                    bool refine = true;
                    if (d.refine_kind == OCTMG_REFINE_NEAR_INTERFACE && l >= d.uniform_level) {
                        double c[3] = {d.lo[0] + ((double)x + 0.5) * w, d.lo[1] + ((double)y + 0.5) * w,
                                       D == 3 ? d.lo[2] + ((double)z + 0.5) * w : 0.0};
                        refine = std::fabs(lsf_host(d, d.lsf_params, c)) < d.refine_width * w;
                    }
                    if (refine) add_children(occ, l, x, y, z);
                }
    }
    balance(occ, D, lmax);
    return finalize(d, occ, out, err);
}

bool adapt_tree(const octmg_geom_desc &d, const Tree &old, const int8_t *flags, Tree *out, std::string *err) {
    if (!check_desc(d, err)) return false;
    const int D = d.dim, lmax = d.max_level;
    std::vector<Occ> occ = empty_occ(D, lmax);
    // the old blocks, and the flags of its leaves in canonical leaf order
    std::vector<std::array<int, 5>> coarsen;  // level, x, y, z, -
    long fi = 0;
    for (size_t il = 0; il < old.lv.size(); il++) {
        const int l = (int)il - old.nsub + 1;
        const TreeLevel &T = old.lv[il];
        for (int b = 0; b < T.nblocks(); b++) {
            const int x = T.pos[3 * b], y = T.pos[3 * b + 1], z = T.pos[3 * b + 2];
            if (l >= 1) occ[l].bits[occ[l].idx(x, y, z)] = 1;
            if (!T.leaf[b]) continue;
            const int f = flags[fi++];
            if (l < 1) continue;
            if (f > 0 && l < lmax) add_children(occ, l, x, y, z);
            if (f < 0 && l > 1 && l > d.uniform_level) coarsen.push_back({l, x, y, z, 0});
        }
    }
    // a parent loses its children only when all of them were leaves flagged
    // for coarsening (and none was refined above)
    std::vector<std::vector<uint8_t>> votes(lmax + 1);
    for (int l = 1; l <= lmax; l++) votes[l].assign(occ[l].bits.size(), 0);
    for (const auto &c : coarsen) votes[c[0] - 1][occ[c[0] - 1].idx(c[1] >> 1, c[2] >> 1, c[3] >> 1)]++;
    const int nch = D == 3 ? 8 : 4;
    for (int l = 2; l <= lmax; l++) {
        const int nb = occ[l - 1].nb, nz = D == 3 ? nb : 1;
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < nb; y++)
                for (int x = 0; x < nb; x++) {
                    if (votes[l - 1][occ[l - 1].idx(x, y, z)] != nch) continue;
                    bool grand = false;  // a refined child keeps the family
                    if (l < lmax)
                        for (int c = 0; c < nch; c++)
                            grand = grand || occ[l + 1].has(2 * (2 * x + (c & 1)), 2 * (2 * y + (c >> 1 & 1)),
                                                            D == 3 ? 2 * (2 * z + (c >> 2)) : 0);
                    if (grand) continue;
                    for (int c = 0; c < nch; c++)
                        occ[l].bits[occ[l].idx(2 * x + (c & 1), 2 * y + (c >> 1 & 1), D == 3 ? 2 * z + (c >> 2) : 0)] = 0;
                }
    }
    balance(occ, D, lmax);
    return finalize(d, occ, out, err);
}

}  // namespace octmg
