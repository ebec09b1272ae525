// Binary64 overlap tests in the frame of particle A (Sec. 2.3).  Their
// operation order is pinned so that every decision is reproducible: products
// are rounded before sums, sums run left to right, nothing is fused.
#pragma once

#include "device_common.hpp"
#include "types.hpp"

namespace hpmc {

// ---------------------------------------------------------------------------
// Convex polygons, separating axes.  z = conj(zA) zB is B's orientation
// relative to A and t = conj(zA) r B's centre in A's frame.  A's edge normals
// are tried with B's vertices mapped into A's frame, then B's edge normals
// with A's vertices mapped into B's frame; the shapes' own projections onto
// their own normals are per-shape constants.  An axis separates when the
// projection intervals are disjoint or touch.
// ---------------------------------------------------------------------------
// One half of the axes: HALF 0 = A's normals with B's vertices mapped into
// A's frame, HALF 1 = B's normals with A's vertices mapped into B's frame.
// True when one of them separates.
template <int NV, int HALF>
__device__ __forceinline__ bool polygon_half_separated64(const SpeciesDev& P, double rx, double ry,
                                                         double cA, double sA, double cB, double sB) {
    // NV > 0: vertex count known at compile time; NV == 0: P.nv at run time
    constexpr int MV = NV > 0 ? NV : kMaxPolyVerts;
    const int nv = NV > 0 ? NV : P.nv;
    const double zc = cA * cB + sA * sB;
    const double zs = cA * sB - sA * cB;
    const double tx = cA * rx + sA * ry;
    const double ty = cA * ry - sA * rx;

    double px[MV], py[MV];
#pragma unroll
    for (int j = 0; j < MV; ++j) {
        if (j < nv) {
            if constexpr (HALF == 0) {
                px[j] = (zc * P.vx[j] - zs * P.vy[j]) + tx;
                py[j] = (zs * P.vx[j] + zc * P.vy[j]) + ty;
            } else {
                const double ux = P.vx[j] - tx;
                const double uy = P.vy[j] - ty;
                px[j] = zc * ux + zs * uy;
                py[j] = zc * uy - zs * ux;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < MV; ++k) {
        if (k < nv) {
            const double nx = P.nx[k], ny = P.ny[k];
            double lo = nx * px[0] + ny * py[0];
            double hi = lo;
#pragma unroll
            for (int j = 1; j < MV; ++j) {
                if (j < nv) {
                    const double p = nx * px[j] + ny * py[j];
                    lo = fmin(lo, p);
                    hi = fmax(hi, p);
                }
            }
            if constexpr (HALF == 0) {
                if (P.pmax[k] <= lo || hi <= P.pmin[k]) return true;
            } else {
                if (hi <= P.pmin[k] || P.pmax[k] <= lo) return true;
            }
        }
    }
    return false;
}

template <int NV>
__device__ __forceinline__ bool polygon_overlap64(const SpeciesDev& P, double rx, double ry,
                                                  double cA, double sA, double cB, double sB) {
    return !polygon_half_separated64<NV, 0>(P, rx, ry, cA, sA, cB, sB) &&
           !polygon_half_separated64<NV, 1>(P, rx, ry, cA, sA, cB, sB);
}

// ---------------------------------------------------------------------------
// Spheropolygons: a core polygon swept by a disk of radius s (Sec. 2.3's
// swept shapes).  Two overlap when the cores overlap (the separating axes
// above) or pass closer than s + s; cores that do not meet are closest at a
// vertex of one and an edge of the other, and a core of one or two vertices
// (a point, a segment) is covered by its edges k -> k+1 all the same.
// Distances are taken in A's frame with B's vertices mapped as in HALF 0.
// ---------------------------------------------------------------------------
// Point p closer than r (r2 = r^2) to segment a-b: nearest point a when the
// projection parameter c1 <= 0, b when c1 >= c2 = |b - a|^2, else the foot of
// the perpendicular at squared distance cross^2 / c2.
__device__ __forceinline__ bool point_segment_close64(double px, double py, double ax, double ay,
                                                      double bx, double by, double r2) {
    const double ex = bx - ax, ey = by - ay;
    const double wx = px - ax, wy = py - ay;
    const double c1 = wx * ex + wy * ey;
    if (c1 <= 0.0) return wx * wx + wy * wy < r2;
    const double c2 = ex * ex + ey * ey;
    if (c1 >= c2) {
        const double dx = px - bx, dy = py - by;
        return dx * dx + dy * dy < r2;
    }
    const double cr = ex * wy - ey * wx;
    return cr * cr < r2 * c2;
}

__device__ __forceinline__ bool polygon_cores_close64(const SpeciesDev& P, double rx, double ry,
                                                      double cA, double sA, double cB, double sB) {
    constexpr int MV = kMaxPolyVerts;
    const int nv = P.nv;
    const double zc = cA * cB + sA * sB;
    const double zs = cA * sB - sA * cB;
    const double tx = cA * rx + sA * ry;
    const double ty = cA * ry - sA * rx;
    const double reach = P.sweep + P.sweep;
    const double r2 = reach * reach;
    // B's vertices in A's frame, in registers (compile-time indices only)
    double bx[MV], by[MV];
#pragma unroll
    for (int j = 0; j < MV; ++j) {
        bx[j] = 0.0;
        by[j] = 0.0;
        if (j < nv) {
            bx[j] = (zc * P.vx[j] - zs * P.vy[j]) + tx;
            by[j] = (zs * P.vx[j] + zc * P.vy[j]) + ty;
        }
    }
    // the uniform loop runs over A's vertex / edge k (scalar reads), the
    // unrolled one over B's
    for (int k = 0; k < nv; ++k) {
        const int k1 = k + 1 < nv ? k + 1 : 0;
        const double ax = P.vx[k], ay = P.vy[k], ax1 = P.vx[k1], ay1 = P.vy[k1];
#pragma unroll
        for (int j = 0; j < MV; ++j) {
            if (j < nv) {
                // A's vertex k against B's edge j -> j+1
                const double bx1 = j + 1 < nv ? bx[j + 1 < MV ? j + 1 : 0] : bx[0];
                const double by1 = j + 1 < nv ? by[j + 1 < MV ? j + 1 : 0] : by[0];
                if (point_segment_close64(ax, ay, bx[j], by[j], bx1, by1, r2)) return true;
                // B's vertex j against A's edge k -> k+1
                if (point_segment_close64(bx[j], by[j], ax, ay, ax1, ay1, r2)) return true;
            }
        }
    }
    return false;
}

__device__ __forceinline__ bool spheropolygon_overlap64(const SpeciesDev& P, double rx, double ry,
                                                        double cA, double sA, double cB, double sB) {
    return polygon_overlap64<0>(P, rx, ry, cA, sA, cB, sB) ||
           polygon_cores_close64(P, rx, ry, cA, sA, cB, sB);
}

// ---------------------------------------------------------------------------
// Convex polyhedra, XenoCollide (minkowski portal refinement; Jacobs 2008,
// Snethen).  D = B - A in A's frame, support S_D(n) = M S_B(M^T n) + t -
// S_A(-n) (Eq. 2, with the centre offset rotated into A's frame), where S_X
// picks the first vertex of largest projection.  v0 = t is interior to D; a
// portal (v1, v2, v3) crossed by the ray from v0 through the origin is found
// and then pushed onto the boundary of D.
// ---------------------------------------------------------------------------
struct V3 { double x, y, z; };

__host__ __device__ inline double dot(const V3& a, const V3& b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__host__ __device__ inline V3 cross(const V3& a, const V3& b) {
    return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__host__ __device__ inline V3 sub(const V3& a, const V3& b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__host__ __device__ inline V3 neg(const V3& a) { return V3{-a.x, -a.y, -a.z}; }
__host__ __device__ inline bool is_zero(const V3& a) { return a.x == 0.0 && a.y == 0.0 && a.z == 0.0; }

struct Minkowski64 {
    Mat3 M;  // B frame -> A frame
    V3 t;    // B's centre in A's frame
};

// Set-up shared by the binary64 and binary32 tests: M = R(conj(qa) qb),
// t = R(qa)^T r.
__host__ __device__ inline Minkowski64 polyhedron_setup64(const V3& r, const Quat& qa, const Quat& qb) {
    Minkowski64 mk;
    const Quat qac{qa.w, -qa.x, -qa.y, -qa.z};
    mk.M = rotation_matrix(qmul(qac, qb));
    const Mat3 ma = rotation_matrix(qa);
    mk.t = V3{(ma.m[0][0] * r.x + ma.m[1][0] * r.y) + ma.m[2][0] * r.z,
              (ma.m[0][1] * r.x + ma.m[1][1] * r.y) + ma.m[2][1] * r.z,
              (ma.m[0][2] * r.x + ma.m[1][2] * r.y) + ma.m[2][2] * r.z};
    return mk;
}

__device__ __forceinline__ V3 support64(const SpeciesDev& P, const Minkowski64& mk, const V3& n) {
    const int nv = P.nv;
    const double(&m)[3][3] = mk.M.m;
    const V3 nb{(m[0][0] * n.x + m[1][0] * n.y) + m[2][0] * n.z,
                (m[0][1] * n.x + m[1][1] * n.y) + m[2][1] * n.z,
                (m[0][2] * n.x + m[1][2] * n.y) + m[2][2] * n.z};
    const V3 na = neg(n);
    int kb = 0, ka = 0;
    double bb = (nb.x * P.vx[0] + nb.y * P.vy[0]) + nb.z * P.vz[0];
    double ba = (na.x * P.vx[0] + na.y * P.vy[0]) + na.z * P.vz[0];
    // four vertices per iteration: their scalar loads are issued together and
    // share one wait (the vertex count is a run-time value)
#pragma unroll 4
    for (int k = 1; k < nv; ++k) {
        const double vx = P.vx[k], vy = P.vy[k], vz = P.vz[k];
        const double pb = (nb.x * vx + nb.y * vy) + nb.z * vz;
        const double pa = (na.x * vx + na.y * vy) + na.z * vz;
        if (pb > bb) { bb = pb; kb = k; }
        if (pa > ba) { ba = pa; ka = k; }
    }
    const double bx = P.vx[kb], by = P.vy[kb], bz = P.vz[kb];
    V3 out{(((m[0][0] * bx + m[0][1] * by) + m[0][2] * bz) + mk.t.x) - P.vx[ka],
           (((m[1][0] * bx + m[1][1] * by) + m[1][2] * bz) + mk.t.y) - P.vy[ka],
           (((m[2][0] * bx + m[2][1] * by) + m[2][2] * bz) + mk.t.z) - P.vz[ka]};
    // spheropolyhedra: each particle's ball adds sweep n/|n| to its support,
    // so the difference gains (sweep + sweep) n/|n| (none for n = 0)
    if (P.sweep > 0.0) {  // uniform per species: plain polyhedra skip it whole
        const double nn = dot(n, n);
        if (nn > 0.0) {
            const double s = (P.sweep + P.sweep) / sqrt(nn);
            out = V3{out.x + s * n.x, out.y + s * n.y, out.z + s * n.z};
        }
    }
    return out;
}

constexpr int kMprMaxIter = 1024;

__device__ __forceinline__ bool polyhedron_mpr64(const SpeciesDev& P, const Minkowski64& mk) {
    const V3 v0 = mk.t;
    if (is_zero(v0)) return true;  // coincident centres

    V3 n = neg(v0);
    V3 v1 = support64(P, mk, n);
    if (dot(v1, n) <= 0.0) return false;
    n = cross(v1, v0);
    if (is_zero(n)) return true;  // origin on the segment v0 -> v1
    V3 v2 = support64(P, mk, n);
    if (dot(v2, n) <= 0.0) return false;
    n = cross(sub(v1, v0), sub(v2, v0));
    if (dot(n, v0) > 0.0) {
        const V3 s = v1;
        v1 = v2;
        v2 = s;
        n = neg(n);
    }

    int iter = 0;
    V3 v3;
    for (;;) {  // portal discovery
        if (++iter > kMprMaxIter) return true;
        v3 = support64(P, mk, n);
        if (dot(v3, n) <= 0.0) return false;
        if (dot(cross(v1, v3), v0) < 0.0) {  // origin outside face (v0, v1, v3)
            v2 = v3;
            n = cross(sub(v1, v0), sub(v3, v0));
            continue;
        }
        if (dot(cross(v3, v2), v0) < 0.0) {  // origin outside face (v0, v3, v2)
            v1 = v3;
            n = cross(sub(v3, v0), sub(v2, v0));
            continue;
        }
        break;
    }

    for (;;) {  // portal refinement
        if (++iter > kMprMaxIter) return true;
        n = cross(sub(v2, v1), sub(v3, v1));
        if (dot(n, v1) >= 0.0) return true;  // origin behind the portal
        const V3 v4 = support64(P, mk, n);
        if (dot(v4, n) <= 0.0) return false;
        const double gap = dot(sub(v4, v3), n);
        if (gap <= 0.0 || gap * gap <= P.tol2 * dot(n, n)) return false;
        const V3 tmp = cross(v4, v0);
        if (dot(v1, tmp) > 0.0) {
            if (dot(v2, tmp) > 0.0)
                v1 = v4;
            else
                v3 = v4;
        } else {
            if (dot(v3, tmp) > 0.0)
                v2 = v4;
            else
                v1 = v4;
        }
    }
}

__device__ __forceinline__ bool polyhedron_overlap64(const SpeciesDev& P, const V3& r, const Quat& qa,
                                                  const Quat& qb) {
    return polyhedron_mpr64(P, polyhedron_setup64(r, qa, qb));
}

}  // namespace hpmc
