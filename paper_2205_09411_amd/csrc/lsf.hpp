// Level-set functions (Sec. 3.1: the interface is the zero contour of f).
//
// One definition serves the device setup (built-in kinds, evaluated inside
// the setup kernels) and the host (refinement test of the tree builder, and
// the whole setup when the level set is a user callback).  Only + - * / sqrt
// and comparisons are used, all correctly rounded, with FMA contraction off
// inside every function, so host and device give the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "octmg.h"

namespace octmg {

__host__ __device__ inline double sqrt_rn(double v) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __dsqrt_rn(v);
#else
    return std::sqrt(v);
#endif
}

// cube root of a >= 0 from + - * / alone: powers of 8 bring a into
// [1/8, 1), six Newton steps from 3/4 on t^3 = m, powers of 2 scale back
__host__ __device__ inline double cbrt_ops(double a) {
    #pragma clang fp contract(off)
    if (!(a > 0.0)) return 0.0;
    int k = 0;
    double m = a;
    while (m >= 1.0) {
        m = m * 0.125;
        ++k;
    }
    while (m < 0.125) {
        m = m * 8.0;
        --k;
    }
    double t = 0.75;
    for (int it = 0; it < 6; ++it) t = (2.0 * t + m / (t * t)) / 3.0;
    for (; k > 0; --k) t = t * 2.0;
    for (; k < 0; ++k) t = t * 0.5;
    return t;
}

// The level set of a geometry.  `params` must be readable where the
// evaluation runs (a device copy inside kernels, the host copy otherwise);
// `fn`/`user` are used on the host only (OCTMG_LSF_CALLBACK).
struct Lsf {
    int kind, n, D;
    const double *params;
    octmg_lsf_fn fn;
    void *user;

    // the sharp shapes of Sec. 4.2 on the (p, q) plane; params
    // [cx, cy, cz, s, r0], in 3D axisymmetric about the z axis through
    // (cx, cy) with p = s (|(x - cx, y - cy)| - r0)
    __host__ __device__ double shape(const double *x) const {
        #pragma clang fp contract(off)
        const double *c = params;
        double p, q;
        if (D == 2) {
            p = c[3] * (x[0] - c[0]);
            q = c[3] * (x[1] - c[1]);
        } else {
            const double ex = x[0] - c[0], ey = x[1] - c[1];
            p = c[3] * (sqrt_rn(ex * ex + ey * ey) - c[4]);
            q = c[3] * (x[2] - c[2]);
        }
        if (kind == OCTMG_LSF_SPHEROID) return sqrt_rn(8.0 * p * p + q * q) - 1.0;
        if (kind == OCTMG_LSF_RHOMBUS) return 8.0 * fabs(p) + fabs(q) - 1.5;
        if (kind == OCTMG_LSF_HEART) {
            const double h = q - cbrt_ops(p * p);
            return p * p + h * h - 1.0;
        }
        return cbrt_ops(p * p) / 0.8 + cbrt_ops(q * q) / 1.5 - 0.8;
    }

    // rod (points within r_rod of segment a-b) and sphere, the nearer surface
    __host__ __device__ double electrodes(const double *x) const {
        #pragma clang fp contract(off)
        const double *q = params;
        double ab[3], t = 0.0, ll = 0.0;
        for (int c = 0; c < 3; ++c) {
            ab[c] = q[3 + c] - q[c];
            t += (x[c] - q[c]) * ab[c];
            ll += ab[c] * ab[c];
        }
        t = t / ll;
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        double d2 = 0.0, s2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double e = x[c] - (q[c] + t * ab[c]), f = x[c] - q[7 + c];
            d2 += e * e;
            s2 += f * f;
        }
        const double rod = sqrt_rn(d2) - q[6], sph = sqrt_rn(s2) - q[10];
        return rod < sph ? rod : sph;
    }

    // built-in kinds; 1 (no interface) for OCTMG_LSF_NONE
    __host__ __device__ double builtin(const double *x) const {
        #pragma clang fp contract(off)
        const double *p = params;
        if (kind == OCTMG_LSF_ELECTRODES) return electrodes(x);
        if (kind >= OCTMG_LSF_SPHEROID && kind <= OCTMG_LSF_ASTROID) return shape(x);
        if (kind == OCTMG_LSF_SPHERES) {
            double best = 0.0;
            for (int m = 0; m < n; m++) {
                double ex = x[0] - p[4 * m], ey = x[1] - p[4 * m + 1];
                double r2 = ex * ex + ey * ey;
                if (D == 3) {
                    double ez = x[2] - p[4 * m + 2];
                    r2 = r2 + ez * ez;
                }
                double v = sqrt_rn(r2) - p[4 * m + 3];
                if (m == 0 || v < best) best = v;
            }
            return best;
        }
        if (kind == OCTMG_LSF_CYLINDER_Z) {
            double ex = x[0] - p[0], ey = x[1] - p[1];
            return sqrt_rn(ex * ex + ey * ey) - p[2];
        }
        return 1.0;
    }

    __host__ __device__ double operator()(const double *x) const {
#if !defined(__HIP_DEVICE_COMPILE__)
        if (kind == OCTMG_LSF_CALLBACK) {
            // the callback sees all three coordinates (z = 0 in 2D)
            double xx[3] = {x[0], x[1], D == 3 ? x[2] : 0.0};
            return fn(xx, user);
        }
#endif
        return builtin(x);
    }
};

}  // namespace octmg
