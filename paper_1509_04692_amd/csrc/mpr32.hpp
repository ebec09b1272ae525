// Certified binary32 XenoCollide for convex polyhedra (mixed precision).
//
// The binary64 test (overlap64.hpp) walks a fixed sequence of decisions: sign
// tests of dot and triple products, the tolerance test, and in every support
// call the choice of the vertex of largest projection.  This version walks
// the same sequence in binary32 and trusts a decision only when it provably
// agrees with the binary64 one.  Both are compared with the exact-arithmetic
// evaluation on the binary64 set-up values (rotation matrix M and centre
// offset t, computed in binary64 exactly as the binary64 test does, and the
// binary64 vertex table): every binary32 vector carries a bound on the
// absolute error of each component, and a decision is certified when its
// binary32 value is farther from zero than the bound of its own error plus
// that of the binary64 evaluation (the latter is at most 2^-29 of the
// former, covered by a relative factor).  With every decision certified the
// two evaluations follow the same branches and pick the same vertices, so
// the binary32 result equals the binary64 one.  Anything uncertain returns
// kMprUncertain and the caller runs the binary64 test.
//
// Error model (u = 2^-24, R the circumradius, |t| < 2R after the
// circumsphere test, every support point within 4R of the origin):
//   * inputs: binary32 casts of M, t and the vertices, relative error u;
//   * support point S_D(n) = M v_b + t - v_a, with the same vertex indices
//     as the exact evaluation: per component within 40 u R (casts 6.5 u R,
//     six roundings of magnitudes <= 4R);
//   * a difference p - q: e_p + e_q + u |p - q|;
//   * a cross product a x b: e_a |b|_1 + e_b |a|_1 + 2u |a|_1 |b|_1;
//   * a dot product a . b: e_a |b|_1 + e_b |a|_1 + 3u |a|_1 |b|_1;
// (1-norms of the binary32 values, enlarged by 3 e to cover the exact
// ones; second-order terms included).  Values that depend on a support call
// only through its projection -- dot(S(n), n), and the gap -- are support
// function values h(n) and do not need the vertex choice certified: the
// chosen vertex is within 2 x (projection rounding) of the maximum, and
// |h(n) - h(n')| <= 4 sqrt(3) R |n - n'|_inf.  A support point that the
// walk keeps as a portal vertex must have its choice certified: the largest
// and second largest projections on each shape differ by more than twice
// their error.  All bounds are doubled (kSlack) to absorb the rounding of the
// bound arithmetic itself and the binary64 evaluation's error.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "types.hpp"

// Observation hooks for a host build of the test harness (empty in the
// library): every certified sign decision's value and error bound, the gap
// test's value and bound, and the vertex pair of every support call.
#ifndef HPMC_MPR32_OBSERVE
#define HPMC_MPR32_OBSERVE(x, e)
#endif
#ifndef HPMC_MPR32_SUPPORT
#define HPMC_MPR32_SUPPORT(ka, kb)
#endif

namespace hpmc {

#define HPMC_HD __host__ __device__ inline

enum : int { kMprNoOverlap = 0, kMprOverlap = 1, kMprUncertain = 2 };

constexpr float kU32 = 0x1p-24f;
#ifndef HPMC_MPR32_SLACK
#define HPMC_MPR32_SLACK 2.0f  // tests build a variant with a shrunken bound
#endif
constexpr float kSlack = HPMC_MPR32_SLACK;
constexpr int kMpr32MaxIter = 1024;

struct F3 {
    float x, y, z;
};

// A binary32 vector and the bound on the error of each of its components.
struct TV {
    F3 v;
    float e;
};

HPMC_HD float norm1(const F3& a) { return (fabsf(a.x) + fabsf(a.y)) + fabsf(a.z); }
HPMC_HD float dotf(const F3& a, const F3& b) { return fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x)); }
HPMC_HD F3 crossf(const F3& a, const F3& b) {
    return F3{fmaf(a.y, b.z, -(a.z * b.y)), fmaf(a.z, b.x, -(a.x * b.z)), fmaf(a.x, b.y, -(a.y * b.x))};
}

HPMC_HD TV tv_sub(const TV& a, const TV& b) {
    const F3 d{a.v.x - b.v.x, a.v.y - b.v.y, a.v.z - b.v.z};
    return TV{d, a.e + b.e + kU32 * norm1(d)};
}

HPMC_HD TV tv_cross(const TV& a, const TV& b) {
    const float a1 = norm1(a.v) + 3.0f * a.e, b1 = norm1(b.v) + 3.0f * b.e;
    const float e = kSlack * (a.e * b1 + b.e * a1 + 2.0f * kU32 * a1 * b1 + 2.0f * a.e * b.e);
    return TV{crossf(a.v, b.v), e};
}

// Error bound of dot(a, b).
HPMC_HD float tv_dot_err(const TV& a, const TV& b) {
    const float a1 = norm1(a.v) + 3.0f * a.e, b1 = norm1(b.v) + 3.0f * b.e;
    return kSlack * (a.e * b1 + b.e * a1 + 3.0f * kU32 * a1 * b1 + 3.0f * a.e * b.e);
}

// Sign of a value with error bound e: +1, -1, or 0 when uncertain.
HPMC_HD int certain_sign(float x, float e) {
    HPMC_MPR32_OBSERVE(x, e);
    return x > e ? 1 : (x < -e ? -1 : 0);
}

// Binary32 copies of the set-up values.
struct Mink32 {
    float m[3][3];  // B frame -> A frame
    TV t;           // B's centre in A's frame (the interior point v0)
};

// Support point of D = B - A in direction n (a TV), with the gap between the
// largest and second largest projection on each shape (for certification of
// the vertex choice).  First vertex of largest projection, as in binary64.
struct Sup32 {
    TV p;
    float sep;   // min over both shapes of (largest - second largest projection)
    float eproj; // bound on the error of each projection against the exact ones
};

HPMC_HD Sup32 support32(const SpeciesDev& P, const Mink32& mk, const TV& n) {
    const int nv = P.nv;
    const float(&m)[3][3] = mk.m;
    const F3 nb{fmaf(m[2][0], n.v.z, fmaf(m[1][0], n.v.y, m[0][0] * n.v.x)),
                fmaf(m[2][1], n.v.z, fmaf(m[1][1], n.v.y, m[0][1] * n.v.x)),
                fmaf(m[2][2], n.v.z, fmaf(m[1][2], n.v.y, m[0][2] * n.v.x))};
    int kb = 0, ka = 0;
    float bb = dotf(nb, F3{P.vx32[0], P.vy32[0], P.vz32[0]});
    float ba = -dotf(n.v, F3{P.vx32[0], P.vy32[0], P.vz32[0]});
    float b2 = -INFINITY, a2 = -INFINITY;
    // two vertices per iteration share one wait for their scalar loads
#pragma unroll 2
    for (int k = 1; k < nv; ++k) {
        const F3 v{P.vx32[k], P.vy32[k], P.vz32[k]};
        const float pb = dotf(nb, v);
        const float pa = -dotf(n.v, v);
        b2 = fmaxf(b2, fminf(pb, bb));
        a2 = fmaxf(a2, fminf(pa, ba));
        if (pb > bb) {
            bb = pb;
            kb = k;
        }
        if (pa > ba) {
            ba = pa;
            ka = k;
        }
    }
    HPMC_MPR32_SUPPORT(ka, kb);
    const float bx = P.vx32[kb], by = P.vy32[kb], bz = P.vz32[kb];
    Sup32 s;
    s.p.v = F3{(fmaf(m[0][2], bz, fmaf(m[0][1], by, m[0][0] * bx)) + mk.t.v.x) - P.vx32[ka],
               (fmaf(m[1][2], bz, fmaf(m[1][1], by, m[1][0] * bx)) + mk.t.v.y) - P.vy32[ka],
               (fmaf(m[2][2], bz, fmaf(m[2][1], by, m[2][0] * bx)) + mk.t.v.z) - P.vz32[ka]};
    const float R = P.R32;
    s.p.e = kSlack * 40.0f * kU32 * R;
    s.sep = fminf(bb - b2, ba - a2);
    // projection of vertex k on B: (M^T n) . v_k, against the exact value with
    // the exact n: 12 u R |n|_1 of rounding plus |M v_k|_1 e_n <= sqrt(3) R e_n
    const float n1 = norm1(n.v) + 3.0f * n.e;
    s.eproj = kSlack * (12.0f * kU32 * R * n1 + 1.7320508f * R * n.e);
    return s;
}

// Error bound of a support-function value dot(S(n), n) (vertex choice not
// needed): rounding 12 u R |n|_1, support point error |n|_1 e_p, choice
// within 2 x (12 + 4) u R |n|_1 of the maximum, Lipschitz term 4 sqrt(3) R e_n.
HPMC_HD float support_value_err(const SpeciesDev& P, const TV& n) {
    const float R = P.R32;
    const float n1 = norm1(n.v) + 3.0f * n.e;
    return kSlack * ((12.0f + 40.0f + 32.0f) * kU32 * R * n1 + 6.9282032f * R * n.e);
}

HPMC_HD bool choice_certified(const Sup32& s) { return s.sep > 2.0f * s.eproj; }

// mk64 (binary64 M and t) must be the values the binary64 test computes.
// Returns kMprNoOverlap / kMprOverlap when certified, else kMprUncertain.
HPMC_HD int polyhedron_overlap32(const SpeciesDev& P, const double (&M)[3][3], const double (&t)[3]) {
    Mink32 mk;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) mk.m[i][j] = (float)M[i][j];
    mk.t.v = F3{(float)t[0], (float)t[1], (float)t[2]};
    // cast error; a component that underflows changes the zero tests below
    mk.t.e = kSlack * kU32 * fmaxf(fmaxf(fabsf(mk.t.v.x), fabsf(mk.t.v.y)), fabsf(mk.t.v.z));
    // coincident or nearly coincident centres go to binary64 (keeps every
    // value far above the binary32 underflow range)
    if (!(norm1(mk.t.v) > 0x1p-20f * P.R32)) return kMprUncertain;
    const TV v0 = mk.t;

    TV n{F3{-v0.v.x, -v0.v.y, -v0.v.z}, v0.e};
    Sup32 s = support32(P, mk, n);
    {
        const int sg = certain_sign(dotf(s.p.v, n.v), support_value_err(P, n));
        if (sg == 0) return kMprUncertain;
        if (sg < 0) return kMprNoOverlap;
    }
    if (!choice_certified(s)) return kMprUncertain;
    TV v1 = s.p;
    n = tv_cross(v1, v0);
    {
        // n == 0 exactly (origin on the segment v0 -> v1) only when certain
        const float big = fmaxf(fmaxf(fabsf(n.v.x), fabsf(n.v.y)), fabsf(n.v.z));
        if (!(big > n.e)) return kMprUncertain;
    }
    s = support32(P, mk, n);
    {
        const int sg = certain_sign(dotf(s.p.v, n.v), support_value_err(P, n));
        if (sg == 0) return kMprUncertain;
        if (sg < 0) return kMprNoOverlap;
    }
    if (!choice_certified(s)) return kMprUncertain;
    TV v2 = s.p;
    n = tv_cross(tv_sub(v1, v0), tv_sub(v2, v0));
    {
        const int sg = certain_sign(dotf(n.v, v0.v), tv_dot_err(n, v0));
        if (sg == 0) return kMprUncertain;
        if (sg > 0) {
            const TV tmp = v1;
            v1 = v2;
            v2 = tmp;
            n.v = F3{-n.v.x, -n.v.y, -n.v.z};
        }
    }

    int iter = 0;
    TV v3;
    for (;;) {  // portal discovery
        if (++iter > kMpr32MaxIter) return kMprUncertain;
        s = support32(P, mk, n);
        {
            const int sg = certain_sign(dotf(s.p.v, n.v), support_value_err(P, n));
            if (sg == 0) return kMprUncertain;
            if (sg < 0) return kMprNoOverlap;
        }
        if (!choice_certified(s)) return kMprUncertain;
        v3 = s.p;
        {
            const TV c = tv_cross(v1, v3);
            const int sg = certain_sign(dotf(c.v, v0.v), tv_dot_err(c, v0));
            if (sg == 0) return kMprUncertain;
            if (sg < 0) {
                v2 = v3;
                n = tv_cross(tv_sub(v1, v0), tv_sub(v3, v0));
                continue;
            }
        }
        {
            const TV c = tv_cross(v3, v2);
            const int sg = certain_sign(dotf(c.v, v0.v), tv_dot_err(c, v0));
            if (sg == 0) return kMprUncertain;
            if (sg < 0) {
                v1 = v3;
                n = tv_cross(tv_sub(v3, v0), tv_sub(v2, v0));
                continue;
            }
        }
        break;
    }

    const float tol = P.tol32;
    for (;;) {  // portal refinement
        if (++iter > kMpr32MaxIter) return kMprUncertain;
        n = tv_cross(tv_sub(v2, v1), tv_sub(v3, v1));
        {
            // binary64: origin behind the portal when dot(n, v1) >= 0
            const int sg = certain_sign(dotf(n.v, v1.v), tv_dot_err(n, v1));
            if (sg == 0) return kMprUncertain;
            if (sg > 0) return kMprOverlap;
        }
        s = support32(P, mk, n);
        const float hv = dotf(s.p.v, n.v);
        const float ehv = support_value_err(P, n);
        {
            const int sg = certain_sign(hv, ehv);
            if (sg == 0) return kMprUncertain;
            if (sg < 0) return kMprNoOverlap;
        }
        {
            // gap = dot(v4 - v3, n) = h(n) - dot(v3, n); binary64 stops when
            // gap <= 0 or gap^2 <= tol^2 |n|^2; continue only when
            // gap > 2 tol |n| for certain
            const TV d = tv_sub(s.p, v3);
            const float gap = dotf(d.v, n.v);
            const float egap = ehv + tv_dot_err(v3, n) + kSlack * 3.0f * kU32 * norm1(d.v) * norm1(n.v);
            const float n1 = norm1(n.v) + 3.0f * n.e;
            HPMC_MPR32_OBSERVE(gap, egap);
            if (gap < -egap) return kMprNoOverlap;
            if (!(gap > egap + 2.0f * tol * n1)) return kMprUncertain;
        }
        if (!choice_certified(s)) return kMprUncertain;
        const TV v4 = s.p;
        const TV c = tv_cross(v4, v0);
        const int s1 = certain_sign(dotf(v1.v, c.v), tv_dot_err(v1, c));
        if (s1 == 0) return kMprUncertain;
        if (s1 > 0) {
            const int s2 = certain_sign(dotf(v2.v, c.v), tv_dot_err(v2, c));
            if (s2 == 0) return kMprUncertain;
            if (s2 > 0)
                v1 = v4;
            else
                v3 = v4;
        } else {
            const int s3 = certain_sign(dotf(v3.v, c.v), tv_dot_err(v3, c));
            if (s3 == 0) return kMprUncertain;
            if (s3 > 0)
                v2 = v4;
            else
                v1 = v4;
        }
    }
}

// Host side: binary32 tables of a polyhedron type.  The circumradius and the
// tolerance are rounded up; the binary32 walk is allowed for circumradii in
// [2^-10, 2^10], where every bound stays far from the binary32 underflow and
// overflow ranges.
inline float round_up_float(double x) {
    float f = (float)x;
    if ((double)f < x) f = std::nextafter(f, INFINITY);
    return f;
}

inline void fill_mpr32_tables(SpeciesDev& P, double tol) {
    for (int k = 0; k < P.nv; ++k) {
        P.vx32[k] = (float)P.vx[k];
        P.vy32[k] = (float)P.vy[k];
        P.vz32[k] = (float)P.vz[k];
    }
    P.R32 = round_up_float(P.R);
    P.tol32 = round_up_float(tol);
    P.mpr32_ok = (P.R >= 0x1p-10 && P.R <= 0x1p10) ? 1 : 0;
}

}  // namespace hpmc
