// Certified binary32 filter for the polygon overlap test.
//
// The mixed-precision mode of the paper computes the min-image separation in
// binary64, casts it to binary32 and trusts the binary32 test (Sec. 2.3).
// Here a binary32 decision is only trusted when it cannot differ from the
// binary64 decision: every projection value computed in binary32 (inputs cast
// from binary64, any operation order, fused or not) lies within
// E32 <= 77 u32 |n| R of the exact value defined by the binary64 inputs, and
// the binary64 evaluation within E64 <= 40 u64 |n| R (u = unit roundoff,
// |n| the longest edge normal, R the circumradius, |r| < 2R after the
// circumsphere test).  The margin M = 256 u32 max|n| R exceeds E32 + E64 by
// more than 3x, covering the rounding of the threshold itself.  An axis is
// certainly separating when its binary32 gap exceeds +M and certainly not when
// it is below -M; anything else makes the pair uncertain, and the caller then
// evaluates it in binary64 exactly as the FP64 path does.
#pragma once

#include "device_common.hpp"
#include "mpr32.hpp"
#include "overlap64.hpp"
#include "types.hpp"

// Observation hook of the certified filters: a host build of the test
// harness defines it to record every binary32 decision value beside its
// error bound; the library's build leaves it empty.
#ifndef HPMC_SAT32_OBSERVE
#define HPMC_SAT32_OBSERVE(half, k, lo, hi)
#endif

namespace hpmc {

enum : int { kNoOverlap = 0, kOverlap = 1, kUncertain = 2 };

// One half of the axes (HALF 0: A's normals, B's vertices in A's frame;
// HALF 1: B's normals, A's vertices in B's frame): kHalfSeparated when one
// axis certainly separates, kHalfOverlaps when every axis certainly does
// not, kHalfUnsure otherwise.
enum : int { kHalfSeparated = 0, kHalfOverlaps = 1, kHalfUnsure = 2 };

template <int NV, int HALF>
__host__ __device__ inline int polygon_half32(const SpeciesDev& P, double rxd, double ryd, double cAd,
                                              double sAd, double cBd, double sBd) {
    // NV > 0: vertex count known at compile time; NV == 0: P.nv at run time
    constexpr int MV = NV > 0 ? NV : kMaxPolyVerts;
    const int nv = NV > 0 ? NV : P.nv;
    const float M = P.sat_margin_scale;
    const float rx = (float)rxd, ry = (float)ryd;
    const float cA = (float)cAd, sA = (float)sAd, cB = (float)cBd, sB = (float)sBd;
    const float zc = fmaf(cA, cB, sA * sB);
    const float zs = fmaf(cA, sB, -(sA * cB));
    const float tx = fmaf(cA, rx, sA * ry);
    const float ty = fmaf(cA, ry, -(sA * rx));

    bool unsure = false;
    float px[MV], py[MV];
#pragma unroll
    for (int j = 0; j < MV; ++j) {
        if (j < nv) {
            if constexpr (HALF == 0) {
                px[j] = fmaf(zc, P.vx32[j], fmaf(-zs, P.vy32[j], tx));
                py[j] = fmaf(zs, P.vx32[j], fmaf(zc, P.vy32[j], ty));
            } else {
                const float ux = P.vx32[j] - tx;
                const float uy = P.vy32[j] - ty;
                px[j] = fmaf(zc, ux, zs * uy);
                py[j] = fmaf(zc, uy, -(zs * ux));
            }
        }
    }
#pragma unroll
    for (int k = 0; k < MV; ++k) {
        if (k < nv) {
            const float nx = P.nx32[k], ny = P.ny32[k];
            float lo = fmaf(nx, px[0], ny * py[0]);
            float hi = lo;
#pragma unroll
            for (int j = 1; j < MV; ++j) {
                if (j < nv) {
                    const float p = fmaf(nx, px[j], ny * py[j]);
                    lo = fminf(lo, p);
                    hi = fmaxf(hi, p);
                }
            }
            const float smax = P.pmax32[k], smin = P.pmin32[k];
            HPMC_SAT32_OBSERVE(HALF, k, lo, hi);
            if (lo >= smax + M || hi <= smin - M) return kHalfSeparated;
            unsure |= !(lo < smax - M && hi > smin + M);
        }
    }
    return unsure ? kHalfUnsure : kHalfOverlaps;
}

// The same decision for a polygon with the rotational symmetry of its own
// vertex count (P.regular): the projections of one shape onto the other's
// normals then differ between normals only by the offset of the centres, so
// the extent is computed once per half (normal 0) and every normal adds its
// offset n_k . t.  Exact symmetry makes this equal to the per-normal
// extents; the tables' measured symmetry defect widens the margin
// (P.sat_margin_regular).  Certification as in polygon_half32.
template <int NV>
__host__ __device__ inline int polygon_overlap32_regular(const SpeciesDev& P, double rxd, double ryd,
                                                         double cAd, double sAd, double cBd, double sBd) {
    constexpr int MV = NV > 0 ? NV : kMaxPolyVerts;
    const int nv = NV > 0 ? NV : P.nv;
    const float M = P.sat_margin_regular;
    const float rx = (float)rxd, ry = (float)ryd;
    const float cA = (float)cAd, sA = (float)sAd, cB = (float)cBd, sB = (float)sBd;
    const float zc = fmaf(cA, cB, sA * sB);
    const float zs = fmaf(cA, sB, -(sA * cB));
    const float tx = fmaf(cA, rx, sA * ry);
    const float ty = fmaf(cA, ry, -(sA * rx));
    const float n0x = P.nx32[0], n0y = P.ny32[0];
    bool unsure = false;
    // A's normals: B's vertices (Z b_j + t) projected; Z^T n_0 . b_j
    {
        const float mx = fmaf(zc, n0x, zs * n0y), my = fmaf(zc, n0y, -(zs * n0x));
        float lo = fmaf(mx, P.vx32[0], my * P.vy32[0]), hi = lo;
#pragma unroll
        for (int j = 1; j < MV; ++j) {
            if (j < nv) {
                const float p = fmaf(mx, P.vx32[j], my * P.vy32[j]);
                lo = fminf(lo, p);
                hi = fmaxf(hi, p);
            }
        }
#pragma unroll
        for (int k = 0; k < MV; ++k) {
            if (k < nv) {
                const float c = fmaf(P.nx32[k], tx, P.ny32[k] * ty);
                const float l = lo + c, h = hi + c;
                const float smax = P.pmax32[k], smin = P.pmin32[k];
                HPMC_SAT32_OBSERVE(0, k, l, h);
                if (l >= smax + M || h <= smin - M) return kNoOverlap;
                unsure |= !(l < smax - M && h > smin + M);
            }
        }
    }
    // B's normals: A's vertices in B's frame, Z^T (a_j - t); (Z n_0) . a_j and
    // the offset -n_k . (Z^T t)
    {
        const float mx = fmaf(zc, n0x, -(zs * n0y)), my = fmaf(zs, n0x, zc * n0y);
        const float ux = fmaf(zc, tx, zs * ty), uy = fmaf(zc, ty, -(zs * tx));
        float lo = fmaf(mx, P.vx32[0], my * P.vy32[0]), hi = lo;
#pragma unroll
        for (int j = 1; j < MV; ++j) {
            if (j < nv) {
                const float p = fmaf(mx, P.vx32[j], my * P.vy32[j]);
                lo = fminf(lo, p);
                hi = fmaxf(hi, p);
            }
        }
#pragma unroll
        for (int k = 0; k < MV; ++k) {
            if (k < nv) {
                const float c = -fmaf(P.nx32[k], ux, P.ny32[k] * uy);
                const float l = lo + c, h = hi + c;
                const float smax = P.pmax32[k], smin = P.pmin32[k];
                HPMC_SAT32_OBSERVE(1, k, l, h);
                if (h <= smin - M || l >= smax + M) return kNoOverlap;
                unsure |= !(h > smin + M && l < smax - M);
            }
        }
    }
    return unsure ? kUncertain : kOverlap;
}

template <int NV>
__host__ __device__ inline int polygon_overlap32(const SpeciesDev& P, double rxd, double ryd, double cAd,
                                                 double sAd, double cBd, double sBd) {
    const int a = polygon_half32<NV, 0>(P, rxd, ryd, cAd, sAd, cBd, sBd);
    if (a == kHalfSeparated) return kNoOverlap;
    const int b = polygon_half32<NV, 1>(P, rxd, ryd, cAd, sAd, cBd, sBd);
    if (b == kHalfSeparated) return kNoOverlap;
    return (a == kHalfUnsure || b == kHalfUnsure) ? kUncertain : kOverlap;
}

// Host side: edge normals, own projections and binary32 copies of a polygon
// type (vertices and R already set).  False unless the vertices are
// counter-clockwise and strictly convex (a swept core of one or two
// vertices, a point or a segment, has no turn to check).
inline bool fill_polygon_tables(SpeciesDev& P) {
    double nmax = 0.0;
    for (int k = 0; k < P.nv; ++k) {
        const int k1 = (k + 1) % P.nv, k2 = (k + 2) % P.nv;
        const double ex = P.vx[k1] - P.vx[k], ey = P.vy[k1] - P.vy[k];
        const double fx = P.vx[k2] - P.vx[k1], fy = P.vy[k2] - P.vy[k1];
        if (P.nv >= 3 && !(ex * fy - ey * fx > 0.0)) return false;
        P.nx[k] = ey;
        P.ny[k] = -ex;
        nmax = std::fmax(nmax, std::sqrt(ey * ey + ex * ex));
    }
    for (int k = 0; k < P.nv; ++k) {
        double lo = 0.0, hi = 0.0;
        for (int j = 0; j < P.nv; ++j) {
            const double p = P.nx[k] * P.vx[j] + P.ny[k] * P.vy[j];
            if (j == 0 || p < lo) lo = p;
            if (j == 0 || p > hi) hi = p;
        }
        P.pmin[k] = lo;
        P.pmax[k] = hi;
        P.vx32[k] = (float)P.vx[k];
        P.vy32[k] = (float)P.vy[k];
        P.nx32[k] = (float)P.nx[k];
        P.ny32[k] = (float)P.ny[k];
        P.pmin32[k] = (float)lo;
        P.pmax32[k] = (float)hi;
    }
    P.sat_margin_scale = (float)(256.0 * 0x1p-24 * nmax * P.R);
    // rotational symmetry of the tables: vertex j and normal k against vertex
    // 0 and normal 0 turned by 2 pi j / nv and 2 pi k / nv; the defect enters
    // every projection of the symmetric filter as an absolute error
    double defect_v = 0.0, defect_n = 0.0;
    for (int k = 0; k < P.nv; ++k) {
        const double ang = 6.283185307179586 * k / P.nv, c = std::cos(ang), s = std::sin(ang);
        defect_v = std::fmax(defect_v, std::hypot(P.vx[k] - (c * P.vx[0] - s * P.vy[0]),
                                                  P.vy[k] - (s * P.vx[0] + c * P.vy[0])));
        defect_n = std::fmax(defect_n, std::hypot(P.nx[k] - (c * P.nx[0] - s * P.ny[0]),
                                                  P.ny[k] - (s * P.nx[0] + c * P.ny[0])));
    }
    const double asym = defect_v * nmax + defect_n * P.R;
    P.regular = asym <= 1e-12 * nmax * P.R ? 1 : 0;
    P.sat_margin_regular = (float)((256.0 * 0x1p-24 * nmax * P.R + 4.0 * asym) * (1.0 + 0x1p-20));
    return true;
}

// Mixed-precision polyhedron test: the binary64 set-up, the certified
// binary32 walk, and the binary64 walk when the former is uncertain.
// Returns the overlap bit | (binary64 used) << 1.
__device__ __forceinline__ int polyhedron_overlap_mixed(const SpeciesDev& P, const V3& r, const Quat& qa,
                                                     const Quat& qb) {
    const Minkowski64 mk = polyhedron_setup64(r, qa, qb);
    if (P.mpr32_ok) {
        const double t[3] = {mk.t.x, mk.t.y, mk.t.z};
        const int d = polyhedron_overlap32(P, mk.M.m, t);
        if (d != kMprUncertain) return d;
    }
    return 2 | (polyhedron_mpr64(P, mk) ? 1 : 0);
}

}  // namespace hpmc
