// Exact polyhedral geodesics by window propagation, one source per wave64.
//
// Method (arXiv 2404.19751, Sec. 2.2 MMP paragraph and Sec. 3.1): a shortest
// path on a triangulated surface is straight in the planar unfolding of the
// faces it crosses and can bend only at saddle or boundary vertices. A
// "window" is an interval [b0, b1] of a half-edge h together with the image
// p of its root (the source, or a bend vertex at distance sg) in h's edge
// frame: rays from p through the interval enter face(h). Processing a window
// unfolds face(h)'s third vertex C, queries the targets in face(h), offers C
// as a bend vertex, and emits at most two child windows on the far edges.
// Windows whose lower bound sg + dist(p, interval) reaches the cutoff are
// dropped: this is the paper's submeshing by the Euclidean lower bound, done
// implicitly (no patch copy).
//
// Bend vertices (pseudo-sources) are re-rooted in distance buckets: whenever
// no window is left, every bend vertex whose distance improved since its last
// launch and lies within `launch_delta` of the smallest such distance is
// launched (a full fan of windows, sg = its distance). Windows of a root
// whose distance has improved since they were made are stale and dropped.
// The result is exact for every pair closer than the cutoff: the optimal
// chain's windows all have lower bound below the pair distance, and the last
// launch of every bend vertex carries its final distance.
//
// Mapping to CDNA4: one wavefront per source (persistent grid, sources taken
// in spatial cell order from eight per-XCD work chunks so each XCD's L2 holds
// one region of the mesh); each lane holds one live window in registers; a
// lane with two children keeps one and pushes the other onto the source's
// window stack with a ballot/popcount compaction; idle lanes pop. Target and
// bend-vertex tables live in LDS; their updates are serialised across lanes
// by a ballot loop (no atomics, deterministic per wave order).
#include <cmath>

#include "gsim_internal.h"

namespace gsim {
namespace {

constexpr int kWave = 64;
constexpr int kMaxCand = 128;
constexpr int kHash = 256;
constexpr int kRootCap = 256;
constexpr int kChunks = 8;

struct WinRec {
    double px, py, b0, b1, sg, c, s;
    int32_t he, root;
};
static_assert(sizeof(WinRec) == 64, "window record is 64 bytes");

struct GeoArgs {
    DevMesh m;
    int n;
    const int32_t *face;
    const double *bary;
    const double *xyz;
    const int64_t *cand_off;
    const int32_t *cand;
    const int32_t *order;
    GeoParams gp;
    GeoOut out;
    WinRec *stack;
    int32_t *work;
    Counters *ctr;
};

struct Lds {
    int32_t tj[kMaxCand], tface[kMaxCand], tnext[kMaxCand];
    double tb[kMaxCand][3];
    double tx3[kMaxCand][3];
    double d1[kMaxCand], d2[kMaxCand], t1x[kMaxCand], t1y[kMaxCand];
    int32_t head[kHash];
    int32_t rkey[kRootCap];
    double rD[kRootCap], rL[kRootCap], rtx[kRootCap], rty[kRootCap];
};

__device__ inline int lane_id() { return threadIdx.x; }
__device__ inline uint64_t lanemask_lt() { return (1ull << threadIdx.x) - 1ull; }
__device__ inline int hash_face(int f) { return (int)(((uint32_t)f * 2654435761u) >> 24) & (kHash - 1); }
__device__ inline int hash_vert(int v) { return (int)(((uint32_t)v * 2246822519u) >> 20) & (kRootCap - 1); }

__device__ inline double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

__device__ inline double seg_dist(double px, double py, double b0, double b1) {
    double dx = px < b0 ? b0 - px : (px > b1 ? px - b1 : 0.0);
    return sqrt(dx * dx + py * py);
}

// first target slot in face f (or -1)
__device__ inline int first_in_face(const Lds &L, int f) {
    int s = L.head[hash_face(f)];
    while (s >= 0 && L.tface[s] != f) s = L.tnext[s];
    return s;
}
__device__ inline int next_in_face(const Lds &L, int s, int f) {
    s = L.tnext[s];
    while (s >= 0 && L.tface[s] != f) s = L.tnext[s];
    return s;
}

// Serialised target update: best distance, its tangent, and the best
// distance among candidates whose direction differs (tie gap).
__device__ inline void target_update(Lds &L, bool ok, int slot, double d, double tx, double ty) {
    uint64_t m = __ballot(ok);
    while (m) {
        int l = __ffsll((unsigned long long)m) - 1;
        if (lane_id() == l) {
            double c1 = L.d1[slot];
            double ax = L.t1x[slot], ay = L.t1y[slot];
            bool differ = !(c1 < INFINITY) || fabs(ax * ty - ay * tx) > 1e-6 || ax * tx + ay * ty < 0.0;
            if (d < c1) {
                if (differ) L.d2[slot] = fmin(L.d2[slot], c1);
                L.d1[slot] = d;
                L.t1x[slot] = tx;
                L.t1y[slot] = ty;
            } else if (differ) {
                L.d2[slot] = fmin(L.d2[slot], d);
            }
        }
        m &= m - 1;
    }
}

// Serialised bend-vertex update (insert or improve).
__device__ inline void root_update(Lds &L, bool ok, int v, double d, double tx, double ty, bool &overflow) {
    uint64_t m = __ballot(ok);
    while (m) {
        int l = __ffsll((unsigned long long)m) - 1;
        if (lane_id() == l) {
            int e = hash_vert(v), probes = 0;
            while (L.rkey[e] >= 0 && L.rkey[e] != v && probes < kRootCap) {
                e = (e + 1) & (kRootCap - 1);
                ++probes;
            }
            if (probes >= kRootCap) {
                overflow = true;
            } else if (L.rkey[e] < 0) {
                L.rkey[e] = v;
                L.rD[e] = d;
                L.rL[e] = INFINITY;
                L.rtx[e] = tx;
                L.rty[e] = ty;
            } else if (d < L.rD[e]) {
                L.rD[e] = d;
                L.rtx[e] = tx;
                L.rty[e] = ty;
            }
        }
        m &= m - 1;
    }
}

struct Win {
    double px, py, b0, b1, sg, c, s;
    int he, root;
};

__device__ inline void push_windows(WinRec *stk, int &sp, int cap, bool want, const Win &w, bool &overflow) {
    uint64_t m = __ballot(want);
    int cnt = __popcll(m);
    if (!cnt) return;
    int r = __popcll(m & lanemask_lt());
    if (want) {
        int pos = sp + r;
        if (pos < cap) {
            WinRec q;
            q.px = w.px; q.py = w.py; q.b0 = w.b0; q.b1 = w.b1; q.sg = w.sg; q.c = w.c; q.s = w.s;
            q.he = w.he; q.root = w.root;
            stk[pos] = q;
        } else {
            overflow = true;
        }
    }
    sp = min(sp + cnt, cap);
}

// Child windows of a window (p, [b0,b1]) on half-edge record R, C's
// intercept txc on the entry edge. Left child: across C->A (stored on R.tp,
// frame origin A, x towards C). Right child: across B->C (stored on R.tn,
// frame origin C, x towards B). `full` = the root lies on the entry edge
// itself (both far edges fully visible).
__device__ inline void children(const HeRec &R, const Win &w, double txc, bool full, double cutoff, Win &cl,
                                bool &hl, Win &cr, bool &hr, int &pruned) {
    const double px = w.px, py = w.py, b0 = w.b0, b1 = w.b1;
    hl = false;
    hr = false;
    if (R.tp >= 0 && (full || b0 < txc)) {
        double ex = R.cx / R.Lp, ey = R.cy / R.Lp;
        double x0, x1;
        if (full) {
            x0 = 0.0;
            x1 = R.Lp;
        } else {
            x0 = b0 <= 0.0 ? 0.0 : R.Lp * (py * b0) / (py * R.cx + R.cy * (b0 - px));
            x1 = b1 >= txc ? R.Lp : R.Lp * (py * b1) / (py * R.cx + R.cy * (b1 - px));
            x0 = fmin(fmax(x0, 0.0), R.Lp);
            x1 = fmin(fmax(x1, 0.0), R.Lp);
        }
        cl.px = ex * px + ey * py;
        cl.py = ex * py - ey * px;
        cl.b0 = x0;
        cl.b1 = x1;
        cl.sg = w.sg;
        cl.c = w.c * ex - w.s * ey;
        cl.s = w.s * ex + w.c * ey;
        cl.he = R.tp;
        cl.root = w.root;
        if (x1 - x0 > 1e-12 * R.Lp) {
            if (w.sg + seg_dist(cl.px, cl.py, x0, x1) < cutoff) hl = true;
            else ++pruned;
        }
    }
    if (R.tn >= 0 && (full || b1 > txc)) {
        double ux = (R.L - R.cx) / R.Ln, uy = -R.cy / R.Ln;
        double x0, x1;
        if (full) {
            x0 = 0.0;
            x1 = R.Ln;
        } else {
            double b = b0;
            x0 = b0 <= txc ? 0.0
                           : R.Ln * ((px - R.cx) * (-py) - (py - R.cy) * (b - px)) /
                                 ((R.L - R.cx) * (-py) + R.cy * (b - px));
            b = b1;
            x1 = b1 >= R.L ? R.Ln
                           : R.Ln * ((px - R.cx) * (-py) - (py - R.cy) * (b - px)) /
                                 ((R.L - R.cx) * (-py) + R.cy * (b - px));
            x0 = fmin(fmax(x0, 0.0), R.Ln);
            x1 = fmin(fmax(x1, 0.0), R.Ln);
        }
        double qx = px - R.cx, qy = py - R.cy;
        cr.px = ux * qx + uy * qy;
        cr.py = ux * qy - uy * qx;
        cr.b0 = x0;
        cr.b1 = x1;
        cr.sg = w.sg;
        cr.c = w.c * ux - w.s * uy;
        cr.s = w.s * ux + w.c * uy;
        cr.he = R.tn;
        cr.root = w.root;
        if (x1 - x0 > 1e-12 * R.Ln) {
            if (w.sg + seg_dist(cr.px, cr.py, x0, x1) < cutoff) hr = true;
            else ++pruned;
        }
    }
}

__global__ __launch_bounds__(kWave) void k_geodesic(GeoArgs a) {
    __shared__ Lds L;
    const int lane = lane_id();
    const double cutoff = a.gp.cutoff;
    const HeRec *__restrict__ he = a.m.he;
    WinRec *stk = a.stack + (size_t)blockIdx.x * a.gp.stack_cap;
    const int chunk0 = blockIdx.x % kChunks;
    int chunk = chunk0, chunks_left = kChunks;

    unsigned long long c_win = 0, c_pruned = 0, c_launch = 0, c_stale = 0, c_limited = 0;

    for (;;) {
        // ---- next source: XCD-local chunk first, then the others
        int idx = -1;
        while (chunks_left > 0) {
            int lo = (int)(((int64_t)a.n * chunk) / kChunks), hi = (int)(((int64_t)a.n * (chunk + 1)) / kChunks);
            int t = 0;
            if (lane == 0) t = atomicAdd(&a.work[chunk], 1);
            t = __shfl(t, 0);
            if (lo + t < hi) {
                idx = lo + t;
                break;
            }
            chunk = (chunk + 1) % kChunks;
            --chunks_left;
        }
        if (idx < 0) break;
        const int src = a.order[idx];
        const int64_t c0 = a.cand_off[src];
        const int nc = (int)(a.cand_off[src + 1] - c0);
        if (nc == 0) continue;
        if (nc > kMaxCand) {
            for (int s = lane; s < nc; s += kWave) {
                a.out.dist[c0 + s] = NAN;
                a.out.flags[c0 + s] = 0;
            }
            if (lane == 0) ++c_limited;
            continue;
        }

        // ---- LDS tables
        for (int e = lane; e < kHash; e += kWave) L.head[e] = -1;
        for (int e = lane; e < kRootCap; e += kWave) L.rkey[e] = -1;
        __syncthreads();
        for (int s = lane; s < nc; s += kWave) {
            int j = a.cand[c0 + s];
            int f = a.face[j];
            L.tj[s] = j;
            L.tface[s] = f;
            for (int d = 0; d < 3; ++d) {
                L.tb[s][d] = a.bary[3 * (int64_t)j + d];
                L.tx3[s][d] = a.xyz[3 * (int64_t)j + d];
            }
            L.d1[s] = INFINITY;
            L.d2[s] = INFINITY;
            L.t1x[s] = 0.0;
            L.t1y[s] = 0.0;
            L.tnext[s] = atomicExch(&L.head[hash_face(f)], s);
        }
        __syncthreads();

        bool overflow = false;
        int sp = 0;
        int pruned = 0;
        unsigned long long nwin = 0;

        // ---- seed from the source (root -1, sg = 0)
        const int fs = a.face[src];
        const double sb[3] = {a.bary[3 * (int64_t)src], a.bary[3 * (int64_t)src + 1], a.bary[3 * (int64_t)src + 2]};
        const HeRec R0 = he[3 * fs];
        const double P[3][2] = {{0.0, 0.0}, {R0.L, 0.0}, {R0.cx, R0.cy}};
        const double sx = sb[1] * P[1][0] + sb[2] * P[2][0], sy = sb[1] * P[1][1] + sb[2] * P[2][1];
        {
            // direct targets in the source face
            int slot = lane < 1 ? first_in_face(L, fs) : -1;
            // one lane walks the (short) chain; other lanes idle
            while (__ballot(slot >= 0)) {
                bool ok = slot >= 0;
                double d = 0, tx = 0, ty = 0;
                if (ok) {
                    double qx = L.tb[slot][1] * P[1][0] + L.tb[slot][2] * P[2][0];
                    double qy = L.tb[slot][1] * P[1][1] + L.tb[slot][2] * P[2][1];
                    double dx = qx - sx, dy = qy - sy;
                    d = sqrt(dx * dx + dy * dy);
                    if (d > 0.0) {
                        tx = dx / d;
                        ty = dy / d;
                    }
                }
                target_update(L, ok, slot, d, tx, ty);
                if (ok) slot = next_in_face(L, slot, fs);
            }
        }
        {
            Win w;
            bool want = false, wantA = false, wantB = false;
            Win wa, wb;
            bool rok = false;
            int rv = 0;
            double rd = 0, rtx = 0, rty = 0;
            if (lane < 3) {
                const int k = lane, h = 3 * fs + k;
                const HeRec R = he[h];
                const double ex = (P[(k + 1) % 3][0] - P[k][0]) / R.L, ey = (P[(k + 1) % 3][1] - P[k][1]) / R.L;
                // bend-vertex candidate: the tail of h
                int v = a.m.T[h];
                if (a.m.vflag[v] & VF_PSEUDO) {
                    double dx = P[k][0] - sx, dy = P[k][1] - sy;
                    rd = sqrt(dx * dx + dy * dy);
                    rok = rd < cutoff;
                    rv = v;
                    rtx = rd > 0 ? dx / rd : 0.0;
                    rty = rd > 0 ? dy / rd : 0.0;
                }
                const double hx = sb[(k + 1) % 3] * R.L + sb[(k + 2) % 3] * R.cx, hy = sb[(k + 2) % 3] * R.cy;
                if (R.twin >= 0) {
                    w.px = R.L - hx;
                    w.py = -hy;
                    w.b0 = 0.0;
                    w.b1 = R.L;
                    w.sg = 0.0;
                    w.c = -ex;
                    w.s = -ey;
                    w.he = R.twin;
                    w.root = -1;
                    if (sb[(k + 2) % 3] > 0.0) {
                        want = seg_dist(w.px, w.py, 0.0, R.L) < cutoff;
                    } else {
                        // source on this edge: the face across contains it as well
                        const HeRec Rt = he[R.twin];
                        w.py = 0.0;
                        double txc = 0.0;
                        children(Rt, w, txc, true, cutoff, wa, wantA, wb, wantB, pruned);
                    }
                }
            }
            root_update(L, rok, rv, rd, rtx, rty, overflow);
            // on-edge sources: targets and third vertex of the face across
            for (int k = 0; k < 3; ++k) {
                bool on = sb[(k + 2) % 3] <= 0.0 && he[3 * fs + k].twin >= 0;
                if (!on) continue;  // wave-uniform
                const HeRec R = he[3 * fs + k];
                const int t = R.twin, g = t / 3, m = t % 3;
                const HeRec Rt = he[t];
                const double ex = (P[(k + 1) % 3][0] - P[k][0]) / R.L, ey = (P[(k + 1) % 3][1] - P[k][1]) / R.L;
                const double c = -ex, s = -ey;
                const double hx = sb[(k + 1) % 3] * R.L + sb[(k + 2) % 3] * R.cx;
                const double ptx = R.L - hx;
                int slot = lane < 1 ? first_in_face(L, g) : -1;
                while (__ballot(slot >= 0)) {
                    bool ok = slot >= 0;
                    double d = 0, tx = 0, ty = 0;
                    if (ok) {
                        double qx = L.tb[slot][(m + 1) % 3] * Rt.L + L.tb[slot][(m + 2) % 3] * Rt.cx;
                        double qy = L.tb[slot][(m + 2) % 3] * Rt.cy;
                        double dx = qx - ptx, dy = qy;
                        d = sqrt(dx * dx + dy * dy);
                        if (d > 0) {
                            dx /= d;
                            dy /= d;
                            tx = c * dx - s * dy;
                            ty = s * dx + c * dy;
                        }
                    }
                    target_update(L, ok, slot, d, tx, ty);
                    if (ok) slot = next_in_face(L, slot, g);
                }
                bool ok = lane == 0 && (Rt.flags & 1);
                double dx = Rt.cx - ptx, dy = Rt.cy;
                double d = sqrt(dx * dx + dy * dy);
                root_update(L, ok && d < cutoff, Rt.opp, d, (c * dx - s * dy) / d, (s * dx + c * dy) / d, overflow);
            }
            push_windows(stk, sp, a.gp.stack_cap, want, w, overflow);
            push_windows(stk, sp, a.gp.stack_cap, wantA, wa, overflow);
            push_windows(stk, sp, a.gp.stack_cap, wantB, wb, overflow);
        }

        // ---- propagation
        bool have = false;
        Win w;
        for (;;) {
            // stack writes by other lanes must be visible before popping
            __syncthreads();
            if (__ballot(overflow)) overflow = true;
            if (overflow) break;
            // refill idle lanes from the stack
            uint64_t need = __ballot(!have);
            int take = min(__popcll(need), sp);
            if (!have) {
                int r = __popcll(need & lanemask_lt());
                if (r < take) {
                    WinRec q = stk[sp - 1 - r];
                    w.px = q.px; w.py = q.py; w.b0 = q.b0; w.b1 = q.b1; w.sg = q.sg; w.c = q.c; w.s = q.s;
                    w.he = q.he; w.root = q.root;
                    have = true;
                }
            }
            sp -= take;
            if (__ballot(have) == 0) {
                // no window anywhere: launch the next bucket of bend vertices
                double mn = INFINITY;
                for (int e = lane; e < kRootCap; e += kWave)
                    if (L.rkey[e] >= 0 && L.rD[e] < L.rL[e] && L.rD[e] < cutoff) mn = fmin(mn, L.rD[e]);
                mn = wave_min(mn);
                if (!(mn < INFINITY)) break;
                const double thr = mn + a.gp.launch_delta;
                for (int base = 0; base < kRootCap; base += kWave) {
                    const int e = base + lane;
                    bool sel = L.rkey[e] >= 0 && L.rD[e] < L.rL[e] && L.rD[e] <= thr && L.rD[e] < cutoff;
                    uint64_t m = __ballot(sel);
                    while (m) {
                        const int el = base + __ffsll((unsigned long long)m) - 1;
                        m &= m - 1;
                        const int v = L.rkey[el];
                        const double D = L.rD[el];
                        const double vtx = L.rtx[el], vty = L.rty[el];
                        __syncthreads();
                        if (lane == 0) L.rL[el] = D;
                        ++c_launch;
                        const int f0 = a.m.fan_off[v], f1 = a.m.fan_off[v + 1];
                        const double vx = a.m.V[3 * (int64_t)v], vy = a.m.V[3 * (int64_t)v + 1],
                                     vz = a.m.V[3 * (int64_t)v + 2];
                        for (int fb = f0; fb < f1; fb += kWave) {
                            const int q = fb + lane;
                            const bool act = q < f1;
                            int h = act ? a.m.fan[q] : 0;
                            const int hn = h - h % 3 + (h % 3 + 1) % 3;
                            HeRec Rh = he[h], Rn = he[hn];
                            Win nw;
                            bool want2 = false;
                            if (act && Rn.twin >= 0) {
                                nw.px = Rn.L - Rn.cx;
                                nw.py = -Rn.cy;
                                nw.b0 = 0.0;
                                nw.b1 = Rn.L;
                                nw.sg = D;
                                nw.c = 1.0;
                                nw.s = 0.0;
                                nw.he = Rn.twin;
                                nw.root = el;
                                want2 = D + seg_dist(nw.px, nw.py, 0.0, Rn.L) < cutoff;
                            }
                            // direct targets in face(h)
                            const int g = h / 3;
                            int slot = act ? first_in_face(L, g) : -1;
                            while (__ballot(slot >= 0)) {
                                bool ok = slot >= 0;
                                double d = 0;
                                if (ok) {
                                    double dx = L.tx3[slot][0] - vx, dy = L.tx3[slot][1] - vy,
                                           dz = L.tx3[slot][2] - vz;
                                    d = D + sqrt(dx * dx + dy * dy + dz * dz);
                                }
                                target_update(L, ok, slot, d, vtx, vty);
                                if (ok) slot = next_in_face(L, slot, g);
                            }
                            // adjacent bend vertices along the two edges at v
                            const int u1 = act ? a.m.T[hn] : 0;  // head of h
                            bool ok1 = act && (a.m.vflag[u1] & VF_PSEUDO) && D + Rh.L < cutoff;
                            root_update(L, ok1, u1, D + Rh.L, vtx, vty, overflow);
                            const int u2 = act ? Rh.opp : 0;
                            bool ok2 = act && (a.m.vflag[u2] & VF_PSEUDO) && D + Rh.Lp < cutoff;
                            root_update(L, ok2, u2, D + Rh.Lp, vtx, vty, overflow);
                            push_windows(stk, sp, a.gp.stack_cap, want2, nw, overflow);
                        }
                    }
                }
                continue;
            }
            nwin += (unsigned long long)__popcll(__ballot(have));
            if (nwin > (unsigned long long)a.gp.max_windows) {
                overflow = true;
                break;
            }

            // ---- process the lane's window
            Win cl, cr;
            bool hl = false, hr = false;
            if (have) {
                if (w.root >= 0 && w.sg > L.rD[w.root]) {
                    have = false;
                    ++c_stale;
                }
            }
            HeRec R;
            double txc = 0.0;
            int f = -1;
            if (have) {
                R = he[w.he];
                f = w.he / 3;
                txc = w.px + (R.cx - w.px) * (-w.py) / (R.cy - w.py);
            }
            const double tol = a.gp.cone_tol;
            // targets in face f
            {
                int slot = have ? first_in_face(L, f) : -1;
                const int k = have ? w.he % 3 : 0;
                while (__ballot(slot >= 0)) {
                    bool ok = false;
                    double d = 0, tx = 0, ty = 0;
                    if (slot >= 0) {
                        double qx = L.tb[slot][(k + 1) % 3] * R.L + L.tb[slot][(k + 2) % 3] * R.cx;
                        double qy = L.tb[slot][(k + 2) % 3] * R.cy;
                        double xq = w.px + (qx - w.px) * (-w.py) / (qy - w.py);
                        double sl = tol * R.L;
                        if (xq >= w.b0 - sl && xq <= w.b1 + sl) {
                            double dx = qx - w.px, dy = qy - w.py;
                            double l = sqrt(dx * dx + dy * dy);
                            d = w.sg + l;
                            ok = d < cutoff;
                            if (w.root < 0) {
                                dx /= l;
                                dy /= l;
                                tx = w.c * dx - w.s * dy;
                                ty = w.s * dx + w.c * dy;
                            } else {
                                tx = L.rtx[w.root];
                                ty = L.rty[w.root];
                            }
                        }
                    }
                    target_update(L, ok, slot, d, tx, ty);
                    if (slot >= 0) slot = next_in_face(L, slot, f);
                }
            }
            // third vertex as a bend vertex
            {
                bool ok = false;
                double d = 0, tx = 0, ty = 0;
                if (have && (R.flags & 1)) {
                    double sl = tol * R.L;
                    if (txc >= w.b0 - sl && txc <= w.b1 + sl) {
                        double dx = R.cx - w.px, dy = R.cy - w.py;
                        double l = sqrt(dx * dx + dy * dy);
                        d = w.sg + l;
                        ok = d < cutoff;
                        if (w.root < 0) {
                            dx /= l;
                            dy /= l;
                            tx = w.c * dx - w.s * dy;
                            ty = w.s * dx + w.c * dy;
                        } else {
                            tx = L.rtx[w.root];
                            ty = L.rty[w.root];
                        }
                    }
                }
                root_update(L, ok, have ? R.opp : 0, d, tx, ty, overflow);
            }
            if (have) children(R, w, txc, false, cutoff, cl, hl, cr, hr, pruned);
            // keep one child in the lane, push the other
            bool push = hl && hr;
            push_windows(stk, sp, a.gp.stack_cap, push, cr, overflow);
            if (have) {
                if (hl) w = cl;
                else if (hr) w = cr;
                else have = false;
            }
        }

        // ---- results
        const int32_t *T = a.m.T;
        const double *p0 = a.m.V + 3 * (int64_t)T[3 * fs], *p1 = a.m.V + 3 * (int64_t)T[3 * fs + 1];
        const double *nn = a.m.fnrm + 3 * (int64_t)fs;
        double ex3[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        double el = sqrt(ex3[0] * ex3[0] + ex3[1] * ex3[1] + ex3[2] * ex3[2]);
        ex3[0] /= el;
        ex3[1] /= el;
        ex3[2] /= el;
        double ey3[3] = {nn[1] * ex3[2] - nn[2] * ex3[1], nn[2] * ex3[0] - nn[0] * ex3[2],
                         nn[0] * ex3[1] - nn[1] * ex3[0]};
        __syncthreads();
        for (int s = lane; s < nc; s += kWave) {
            const int64_t o = c0 + s;
            double d = L.d1[s];
            uint8_t fl = 0;
            if (__ballot(overflow)) d = NAN;
            if (L.d2[s] - d <= a.gp.tie_rel * d) fl |= GSIM_PAIR_TIE_BIT;
            if (d == 0.0) fl |= GSIM_PAIR_ZERO_BIT;
            a.out.dist[o] = d;
            a.out.flags[o] = fl;
            for (int q = 0; q < 3; ++q) a.out.tan[3 * o + q] = L.t1x[s] * ex3[q] + L.t1y[s] * ey3[q];
        }
        c_win += nwin;
        c_pruned += (unsigned long long)pruned;
        if (__ballot(overflow)) ++c_limited;
        __syncthreads();
    }
    // counters: lane sums (pruned is per lane; others wave-uniform)
    unsigned long long pr = c_pruned;
    for (int o = 32; o > 0; o >>= 1) pr += __shfl_xor(pr, o);
    if (lane == 0) {
        atomicAdd(&a.ctr->windows, c_win);
        atomicAdd(&a.ctr->pruned, pr);
        atomicAdd(&a.ctr->launches, c_launch);
        atomicAdd(&a.ctr->limited, c_limited);
    }
    unsigned long long st = c_stale;
    for (int o = 32; o > 0; o >>= 1) st += __shfl_xor(st, o);
    if (lane == 0) atomicAdd(&a.ctr->stale, st);
}

}  // namespace

hipError_t launch_geodesic(const DevMesh &m, int n, const int32_t *face, const double *bary, const double *xyz,
                           const PrefilterBufs &pb, const GeoParams &gp, GeoOut out, char *stack_mem,
                           int32_t nslots, int32_t *work_ctr, Counters *ctr, bool fp32, hipStream_t s) {
    (void)fp32;
    GeoArgs a;
    a.m = m;
    a.n = n;
    a.face = face;
    a.bary = bary;
    a.xyz = xyz;
    a.cand_off = pb.cand_off;
    a.cand = pb.cand;
    a.order = pb.order;
    a.gp = gp;
    a.out = out;
    a.stack = reinterpret_cast<WinRec *>(stack_mem);
    a.work = work_ctr;
    a.ctr = ctr;
    hipLaunchKernelGGL(k_geodesic, dim3(nslots), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

size_t window_record_bytes() { return sizeof(WinRec); }

}  // namespace gsim
