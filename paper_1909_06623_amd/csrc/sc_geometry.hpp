// sc_geometry.hpp -- minimum separation of two rigid cores (section 3.1:
// Phi is the minimal separation distance of a pair, negative on overlap).
// A sphere's core is its centre; a spherocylinder's core is the segment
// c + s p, |s| <= h; both are swept by their radius R.
#pragma once

#include "sc_common.hpp"

namespace sc {

struct PBox {
    double len[3];
    int periodic;
};

struct PairGeo {
    double phi;
    V3 n;
    double s, t;
    int flags;  // bit 0: parallel rule, bit 1: zero distance
};

__device__ __forceinline__ double clampd(double x, double lo, double hi) {
    return x < lo ? lo : (x > hi ? hi : x);
}

// Minimum-image displacement c_j - c_i.
__device__ __forceinline__ V3 min_image(V3 ci, V3 cj, const PBox &b) {
    V3 r = cj - ci;
    if (b.periodic) {
        r.x = r.x - b.len[0] * rint(r.x / b.len[0]);
        r.y = r.y - b.len[1] * rint(r.y / b.len[1]);
        r.z = r.z - b.len[2] * rint(r.z / b.len[2]);
    }
    return r;
}

// Closest points of the two cores c_i + s p_i (|s| <= hi) and c_j + t p_j
// (|t| <= hj), r = c_j - c_i. A sphere's core is its centre (h = 0).
__device__ __forceinline__ int closest_st(V3 r, V3 pi, double hi, V3 pj, double hj,
                                          double &s, double &t) {
    s = 0.0;
    t = 0.0;
    if (hi > 0.0 && hj > 0.0) {
        const double b = dot(pi, pj), c = dot(pi, r), f = dot(pj, r);
        const V3 x = cross(pi, pj);
        if (dot(x, x) < 1e-12) {
            // parallel axes: midpoint of the overlap of the projections on
            // p_i, else the end of i facing j
            const double ab = fabs(b);
            const double lo = fmax(-hi, c - hj * ab), up = fmin(hi, c + hj * ab);
            const double s0 = lo <= up ? 0.5 * (lo + up) : (c > 0.0 ? hi : -hi);
            t = clampd(b * s0 - f, -hj, hj);
            s = clampd(c + b * t, -hi, hi);
            return 1;
        }
        s = clampd((c - b * f) / (1.0 - b * b), -hi, hi);
        t = b * s - f;
        if (t < -hj || t > hj) {
            t = t < -hj ? -hj : hj;
            s = clampd(c + b * t, -hi, hi);
        }
    } else if (hj > 0.0) {
        t = clampd(-dot(pj, r), -hj, hj);
    } else if (hi > 0.0) {
        s = clampd(dot(pi, r), -hi, hi);
    }
    return 0;
}

__device__ __forceinline__ PairGeo pair_geo(V3 r, V3 pi, double Ri, double hi, V3 pj,
                                            double Rj, double hj) {
    PairGeo G;
    G.flags = closest_st(r, pi, hi, pj, hj, G.s, G.t);
    const V3 d = v3(r.x + G.t * pj.x - G.s * pi.x, r.y + G.t * pj.y - G.s * pi.y,
                    r.z + G.t * pj.z - G.s * pi.z);
    const double dist = sqrt(dot(d, d));
    if (dist > 0.0) {
        G.n = v3(d.x / dist, d.y / dist, d.z / dist);
    } else {
        G.n = v3(1.0, 0.0, 0.0);
        G.flags |= 2;
    }
    G.phi = dist - Ri - Rj;
    return G;
}

}  // namespace sc
