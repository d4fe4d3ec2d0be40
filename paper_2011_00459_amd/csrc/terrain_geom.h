// terrain_geom.h -- device geometry shared by the step's kernels and the
// macroscale kernels: the rotation of a pose's quaternion and the distance of
// a sphere to a boundary shape (plane, oriented box, heightfield), both in
// FP64 with a fixed operation order.
#ifndef TERRAIN_GEOM_H
#define TERRAIN_GEOM_H

#include <hip/hip_runtime.h>

#include "terrain_internal.h"

namespace trk {

// Rotation matrix of a unit quaternion (w, x, y, z), row-major.  The
// operation order is fixed: box and plane predicates depend on it bitwise.
__device__ inline void quat_to_R(const double* q, double* R)
{
#pragma clang fp contract(off)
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

struct ShapeHit {
    double delta;
    double n[3];
};

// Sphere against a boundary shape (world data of the step).  Returns true on
// contact; fills overlap and the normal (shape -> particle) when hit != NULL.
__device__ inline bool shape_touch(const ShapeDev& S, const float* hf, double x, double y, double z, double r,
                                   double kappa_c, ShapeHit* hit)
{
#pragma clang fp contract(off)
    double Rr = r + (kappa_c > 0.0 ? kappa_c * (2.0 * r) : 0.0);
    if (S.type == TR_PLANE) {
        double sd = ((S.wn[0] * x + S.wn[1] * y) + S.wn[2] * z) - S.wd;
        if (!(sd < 0.0 || sd * sd < Rr * Rr)) return false;
        if (hit) {
            hit->delta = r - sd;
            hit->n[0] = S.wn[0]; hit->n[1] = S.wn[1]; hit->n[2] = S.wn[2];
        }
        return true;
    }
    if (S.type == TR_BOX) {
        const double* R = S.R;
        double dx = x - S.wc[0], dy = y - S.wc[1], dz = z - S.wc[2];
        double l[3], q[3];
        bool inside = true;
        for (int k = 0; k < 3; ++k) {
            l[k] = (R[0 * 3 + k] * dx + R[1 * 3 + k] * dy) + R[2 * 3 + k] * dz;
            q[k] = l[k];
            if (q[k] > S.half[k]) { q[k] = S.half[k]; inside = false; }
            if (q[k] < -S.half[k]) { q[k] = -S.half[k]; inside = false; }
        }
        if (inside) {
            if (hit) {
                int kb = 0;
                double pb = S.half[0] - fabs(l[0]);
                for (int k = 1; k < 3; ++k) {
                    double pk = S.half[k] - fabs(l[k]);
                    if (pk < pb) { pb = pk; kb = k; }
                }
                double sg = l[kb] >= 0.0 ? 1.0 : -1.0;
                for (int k = 0; k < 3; ++k) hit->n[k] = sg * R[k * 3 + kb];
                hit->delta = r + pb;
            }
            return true;
        }
        double e0 = l[0] - q[0], e1 = l[1] - q[1], e2 = l[2] - q[2];
        double d2 = (e0 * e0 + e1 * e1) + e2 * e2;
        if (!(d2 < Rr * Rr)) return false;
        if (hit) {
            double dist = sqrt(d2);
            double nl[3] = {e0 / dist, e1 / dist, e2 / dist};
            for (int k = 0; k < 3; ++k) hit->n[k] = (R[k * 3 + 0] * nl[0] + R[k * 3 + 1] * nl[1]) + R[k * 3 + 2] * nl[2];
            hit->delta = r - dist;
        }
        return true;
    }
    if (S.type == TR_HEIGHTFIELD) {
        double fx = (x - S.ox) * S.inv_l0;
        double fy = (y - S.oy) * S.inv_l0;
        double fi = floor(fx), fj = floor(fy);
        if (fi < 0.0) fi = 0.0;
        if (fi > (double)(S.nx - 2)) fi = (double)(S.nx - 2);
        if (fj < 0.0) fj = 0.0;
        if (fj > (double)(S.ny - 2)) fj = (double)(S.ny - 2);
        int i = (int)fi, j = (int)fj;
        double t = fx - fi, u = fy - fj;
        const float* h = hf + S.hf_off;
        double h00 = h[j * S.nx + i], h10 = h[j * S.nx + i + 1];
        double h01 = h[(j + 1) * S.nx + i], h11 = h[(j + 1) * S.nx + i + 1];
        double hh = (h00 * (1.0 - t) + h10 * t) * (1.0 - u) + (h01 * (1.0 - t) + h11 * t) * u;
        double hx = ((h10 - h00) * (1.0 - u) + (h11 - h01) * u) * S.inv_l0;
        double hy = ((h01 - h00) * (1.0 - t) + (h11 - h10) * t) * S.inv_l0;
        double dz = z - hh;
        double m2 = (1.0 + hx * hx) + hy * hy;
        if (!(dz < 0.0 || dz * dz < (Rr * Rr) * m2)) return false;
        if (hit) {
            double nz = 1.0 / sqrt(m2);
            hit->n[0] = -hx * nz; hit->n[1] = -hy * nz; hit->n[2] = nz;
            hit->delta = r - dz * nz;
        }
        return true;
    }
    return false;
}

}  // namespace trk

#endif
