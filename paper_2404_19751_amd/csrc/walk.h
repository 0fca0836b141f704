#pragma once
// The shift (arXiv 2404.19751, Sec. 3.2): move each particle by its
// displacement along a straight path across faces. Exit edges are found in
// barycentric coordinates (the rate of change of each coordinate along the
// unit direction); at every crossed edge the particle moves into the face
// across it and the direction and the velocity are rotated about the edge
// axis into the new face's plane (parallel transport). A path through a
// vertex leaves along the straightest direction (Polthier-Schmies: equal
// angle on both sides, i.e. half the vertex's angle sum). At a boundary edge
// the remaining displacement is reflected in the face plane; at a boundary
// vertex it is reversed. A particle whose displacement or velocity is not
// finite is left where it is and flagged.
//
// One lane per particle, FP64 throughout; the face-crossing loop is
// latency-bound on the face/vertex records, which stay in L2.
//
// Shared by the walk and update kernels and by the cutoff kernel, which
// moves each source particle as soon as its neighbour row is complete.
#include <cmath>

#include "gsim_internal.h"
#include "particle_ops.h"

namespace gsim {

constexpr int kWalkCap = 10000;
constexpr double kVertexTol = 1e-12;  // x mean edge: exit parameters this close meet at a vertex
constexpr double kNearTol = 1e-9;     // x mean edge: a pass this close to a vertex is flagged

struct d3 {
    double x, y, z;
};
__device__ inline d3 ld3(const double *p) { return {p[0], p[1], p[2]}; }
__device__ inline d3 operator-(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline d3 operator+(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline d3 operator*(double s, d3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline d3 cross(d3 a, d3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ inline d3 unit(d3 a) { return (1.0 / sqrt(dot(a, a))) * a; }

struct WalkCounts {
    unsigned cross_n, vhit, bhit, cap, near, nonfinite;
};

__device__ inline bool finite3(d3 a) { return isfinite(a.x) && isfinite(a.y) && isfinite(a.z); }

// Walk one particle (face f, barycentrics b) by displacement D, carrying the
// velocity v along (when hv). D and v are projected onto f's plane first.
__device__ inline void walk_one(const DevMesh &m, int &f, double b[3], d3 D, d3 &v, bool hv, WalkCounts &wc,
                                uint8_t &fl) {
    if (!finite3(D) || (hv && !finite3(v))) {
        // a non-finite force, displacement or velocity: the particle stays
        wc.nonfinite = 1;
        fl |= PF_NONFINITE;
        return;
    }
    d3 nf = ld3(m.fnrm + 3 * (int64_t)f);
    D = D - dot(D, nf) * nf;
    if (hv) v = v - dot(v, nf) * nf;
    double rem = sqrt(dot(D, D));
    unsigned &cross_n = wc.cross_n, &vhit = wc.vhit, &bhit = wc.bhit, &cap = wc.cap, &near = wc.near;
    const double lbar = m.mean_edge;
    if (rem > 0.0) {
        d3 u = (1.0 / rem) * D;
        int excl = -1;   // slot whose edge was just crossed/reflected: not an exit
        int onlyk = -1;  // sitting on the vertex of this slot: only its opposite edge is an exit
        // an edge crossing leaves the direction (and velocity) as components
        // along the crossed edge te and across it; they are turned into the
        // new face's plane once its record, normal included, has arrived
        bool turn = false;
        d3 te = {0.0, 0.0, 0.0};
        double tue = 0.0, tum = 0.0, tve = 0.0, tvm = 0.0;
        for (int it = 0;; ++it) {
            // the face's vertices in slot order (one record: no dependent
            // load through the vertex indices)
            const double *fp = m.fpos + 18 * (int64_t)f;
            d3 P[3] = {ld3(fp), ld3(fp + 3), ld3(fp + 6)};
            nf = ld3(m.fnrm + 3 * (int64_t)f);
            // the faces across the three edges, loaded with the face so that
            // a crossing waits for the next face's record only
            const int32_t *tp = m.twin + 3 * (int64_t)f;
            const int tw0 = tp[0], tw1 = tp[1], tw2 = tp[2];
            if (turn) {
                const d3 mi = cross(te, nf);  // pointing into this face, away from the crossed edge
                u = tue * te + tum * mi;
                if (hv) v = tve * te + tvm * mi;
                turn = false;
            }
            if (it >= kWalkCap) {
                cap = 1;
                fl |= 4;
                break;
            }
            double twoA = sqrt(dot(cross(P[1] - P[0], P[2] - P[0]), cross(P[1] - P[0], P[2] - P[0])));
            // the edge opposite each slot, from its next to its previous vertex
            const d3 E0 = P[2] - P[1], E1 = P[0] - P[2], E2 = P[1] - P[0];
            double rate[3], s[3];
            int k1 = -1, k2 = -1;
            for (int k = 0; k < 3; ++k) {
                // gradient of b_k: in-plane normal of the opposite edge, pointing to vertex k
                d3 g = cross(nf, k == 0 ? E0 : k == 1 ? E1 : E2);
                rate[k] = dot(u, g) / twoA;
                bool allowed = (onlyk < 0 || k == onlyk) && k != excl;
                s[k] = (allowed && rate[k] < 0.0) ? fmax(-b[k] / rate[k], 0.0) : INFINITY;
            }
            for (int k = 0; k < 3; ++k)
                if (k1 < 0 || s[k] < s[k1]) k1 = k;
            for (int k = 0; k < 3; ++k)
                if (k != k1 && (k2 < 0 || s[k] < s[k2])) k2 = k;
            const double s1 = s[k1], s2 = s[k2];
            if (!(rem > s1)) {
                for (int k = 0; k < 3; ++k) b[k] += rem * rate[k];
                break;
            }
            const double gap = s2 - s1;
            if (gap <= kVertexTol * lbar) {
                // through the vertex where b[k1] and b[k2] vanish together
                const int ws = 3 - k1 - k2;
                const int wv = m.T[3 * (int64_t)f + ws];
                rem -= s1;
                ++vhit;
                fl |= 1;
                if (m.vflag[wv] & VF_BOUNDARY) {
                    u = -1.0 * u;
                    v = -1.0 * v;
                    b[0] = b[1] = b[2] = 0.0;
                    b[ws] = 1.0;
                    onlyk = ws;
                    excl = -1;
                    continue;
                }
                // polar angle (around wv) of the direction back along the path
                const int hin = 3 * f + ws;
                const int a0 = m.fan_off[wv], a1 = m.fan_off[wv + 1];
                double acc = 0.0;
                for (int a = a0; a < a1 && m.fan[a] != hin; ++a) acc += m.corner[m.fan[a]];
                const int hn = hin - hin % 3 + (hin % 3 + 1) % 3;
                d3 e1 = unit(ld3(m.V + 3 * (int64_t)m.T[hn]) - ld3(m.V + 3 * (int64_t)wv));
                d3 back = -1.0 * u;
                double ang = atan2(dot(cross(e1, back), nf), dot(e1, back));
                ang = fmin(fmax(ang, 0.0), m.corner[hin]);
                const double Theta = m.theta[wv];
                double phi = fmod(acc + ang + 0.5 * Theta, Theta);
                // velocity as an angle from the direction of travel
                double vmag = sqrt(dot(v, v)), psi = 0.0;
                if (hv && vmag > 0.0) psi = atan2(dot(cross(u, v), nf), dot(u, v));
                int hout = m.fan[a1 - 1];
                double base = 0.0, run = 0.0;
                for (int a = a0; a < a1; ++a) {
                    double c = m.corner[m.fan[a]];
                    if (phi < run + c) {
                        hout = m.fan[a];
                        base = run;
                        break;
                    }
                    run += c;
                    base = run - c;
                }
                double gam = fmin(fmax(phi - base, 0.0), m.corner[hout]);
                const int g = hout / 3;
                const int ho = hout - hout % 3 + (hout % 3 + 1) % 3;
                d3 ng = ld3(m.fnrm + 3 * (int64_t)g);
                d3 e0 = unit(ld3(m.V + 3 * (int64_t)m.T[ho]) - ld3(m.V + 3 * (int64_t)wv));
                d3 e0p = cross(ng, e0);
                double sg, cg;
                sincos(gam, &sg, &cg);
                u = cg * e0 + sg * e0p;
                if (hv && vmag > 0.0) {
                    double sp, cp;
                    sincos(psi, &sp, &cp);
                    v = vmag * (cp * u + sp * cross(ng, u));
                }
                f = g;
                b[0] = b[1] = b[2] = 0.0;
                b[hout % 3] = 1.0;
                onlyk = hout % 3;
                excl = -1;
                continue;
            }
            if (gap <= kNearTol * lbar) {
                ++near;
                fl |= 2;
            }
            // cross the edge opposite slot k1
            for (int k = 0; k < 3; ++k) b[k] += s1 * rate[k];
            b[k1] = 0.0;
            rem -= s1;
            const int hk = (k1 + 1) % 3;
            d3 e = unit(k1 == 0 ? E0 : k1 == 1 ? E1 : E2);
            d3 mo = cross(e, nf);  // in-plane normal of the edge, pointing out of f
            const int tw = hk == 0 ? tw0 : hk == 1 ? tw1 : tw2;
            if (tw < 0) {
                ++bhit;
                fl |= 8;
                u = u - 2.0 * dot(u, mo) * mo;
                v = v - 2.0 * dot(v, mo) * mo;
                excl = k1;
                onlyk = -1;
                continue;
            }
            ++cross_n;
            const int g = tw / 3, q = tw % 3;
            double nb[3];
            nb[q] = b[(k1 + 2) % 3];
            nb[(q + 1) % 3] = b[(k1 + 1) % 3];
            nb[(q + 2) % 3] = 0.0;
            te = e;
            tue = dot(u, e);
            tum = dot(u, mo);
            if (hv) {
                tve = dot(v, e);
                tvm = dot(v, mo);
            }
            turn = true;
            f = g;
            b[0] = nb[0];
            b[1] = nb[1];
            b[2] = nb[2];
            excl = (q + 2) % 3;
            onlyk = -1;
        }
    }
}

// The walk of particle i by D (the velocity v carried along) and the store
// of its new state into (face_o, bary_o, vel_o), which may be the arrays the
// state was read from. Returns the particle's PF_* flags; wc receives the
// walk's counts.
__device__ inline uint8_t walk_store(const SurfDesc &sd, int i, int f, const double D[3], d3 v, int32_t *face_o,
                                     double *bary_o, double *vel_o, WalkCounts &wc) {
    double b[3] = {sd.bary[3 * i], sd.bary[3 * i + 1], sd.bary[3 * i + 2]};
    wc = WalkCounts{0, 0, 0, 0, 0, 0};
    uint8_t fl = 0;
    walk_one(sd.m, f, b, d3{D[0], D[1], D[2]}, v, true, wc, fl);
    face_o[i] = f;
    bary_o[3 * i] = b[0];
    bary_o[3 * i + 1] = b[1];
    bary_o[3 * i + 2] = b[2];
    vel_o[3 * i] = v.x;
    vel_o[3 * i + 1] = v.y;
    vel_o[3 * i + 2] = v.z;
    if (sd.wflags) sd.wflags[i] = fl;
    return fl;
}

// One time step of particle i from its force F (Sec. 2.1 integrators other
// than FIRE): overdamped or Brownian displacement, or velocity Verlet in
// leapfrog form (unit masses: the stored velocity is v_{k-1/2}; kick by
// dt F(x_k), drift by dt v_{k+1/2}); then the walk. Returns the particle's
// PF_* flags; wc receives the walk's counts.
__device__ inline uint8_t move_particle(const SurfDesc &sd, int i, const double F[3], int32_t *face_o,
                                        double *bary_o, double *vel_o, WalkCounts &wc) {
    const int f = sd.face[i];
    d3 v = ld3(sd.vel + 3 * (int64_t)i);
    double D[3];
    if (sd.ikind == 3) {
        v = v + sd.dt * d3{F[0], F[1], F[2]};
        D[0] = sd.dt * v.x;
        D[1] = sd.dt * v.y;
        D[2] = sd.dt * v.z;
    } else {
        displacement(sd.m, f, i, F, sd.ikind, sd.dt, sd.mobility, sd.kT, sd.friction, sd.seed, *sd.step, D);
    }
    return walk_store(sd, i, f, D, v, face_o, bary_o, vel_o, wc);
}

}  // namespace gsim
