// Window records and helpers shared by the geodesic kernels (cutoff and
// all-pairs): the window itself, its stack records, the per-half-edge
// unfolding record in the working precision, the bend-vertex table, the
// two-level window stack, and the child intervals on the two far edges of
// a face (arXiv 2404.19751, Sec. 2.2 MMP paragraph: rays from a pseudo-source
// image through an interval of an edge, continued across faces).
#pragma once
#include <cmath>

#include "gsim_internal.h"

namespace gsim {
namespace wnd {

constexpr int kWave = 64;
// bend vertices whose fans one launch step flattens over the lanes
constexpr int kLaunchChunk = 256;

template <typename R>
struct Win {
    R px, py, b0, b1, sg, c, s;
    int he, root;
};

// stack records: 64 bytes (FP64) / 32 bytes (FP32). A window of a bend
// vertex takes its tangent from the vertex, not from its own frame rotation
// (c, s), so the FP32 record keeps the bend vertex in the slot of c instead;
// a source window has sg = 0, so the FP32 record keeps its root (-1 - the
// source's place in a group) in the slot of sg.
struct Rec64 {
    double v[7];
    int32_t he, root;
};
struct Rec32 {
    float v[7];   // px, py, b0, b1, then the root's bits, c, s (source windows) or sg, the root's bits, 0
    uint32_t hr;  // he | (1 << 31) for a window of a bend vertex
};
static_assert(sizeof(Rec64) == 64 && sizeof(Rec32) == 32, "stack record sizes");
template <typename R>
struct RecOf;
template <>
struct RecOf<double> {
    using T = Rec64;
};
template <>
struct RecOf<float> {
    using T = Rec32;
};

__device__ inline void store_rec(Rec64 &q, const Win<double> &w) {
    q.v[0] = w.px; q.v[1] = w.py; q.v[2] = w.b0; q.v[3] = w.b1; q.v[4] = w.sg; q.v[5] = w.c; q.v[6] = w.s;
    q.he = w.he;
    q.root = w.root;
}
__device__ inline void load_rec(const Rec64 &q, Win<double> &w) {
    w.px = q.v[0]; w.py = q.v[1]; w.b0 = q.v[2]; w.b1 = q.v[3]; w.sg = q.v[4]; w.c = q.v[5]; w.s = q.v[6];
    w.he = q.he;
    w.root = q.root;
}
__device__ inline void store_rec(Rec32 &q, const Win<float> &w) {
    const bool rooted = w.root >= 0;
    q.v[0] = w.px; q.v[1] = w.py; q.v[2] = w.b0; q.v[3] = w.b1;
    q.v[4] = rooted ? w.sg : __int_as_float(w.root);
    q.v[5] = rooted ? __int_as_float(w.root) : w.c;
    q.v[6] = rooted ? 0.0f : w.s;
    q.hr = (uint32_t)w.he | (rooted ? 0x80000000u : 0u);
}
__device__ inline void load_rec(const Rec32 &q, Win<float> &w) {
    const bool rooted = (q.hr >> 31) != 0;
    w.px = q.v[0]; w.py = q.v[1]; w.b0 = q.v[2]; w.b1 = q.v[3];
    w.sg = rooted ? q.v[4] : 0.0f;
    w.c = rooted ? 1.0f : q.v[5];
    w.s = rooted ? 0.0f : q.v[6];
    w.he = (int)(q.hr & 0x7fffffffu);
    w.root = __float_as_int(rooted ? q.v[5] : q.v[4]);
}

// half-edge record in the working precision
template <typename R>
struct He {
    R L, cx, cy, Lp, Ln, ex, ey, ux, uy;
    int tn, tp, opp;
    bool pseudo;
};
__device__ inline He<double> load_he(const DevMesh &m, int h, double) {
    const HeRec r = m.he[h];
    return {r.L, r.cx, r.cy, r.Lp, r.Ln, r.ex, r.ey, r.ux, r.uy, r.tn, r.tp, r.opp_flags >> 1, (r.opp_flags & 1) != 0};
}
__device__ inline He<float> load_he(const DevMesh &m, int h, float) {
    const HeRecF r = m.hef[h];
    return {r.L, r.cx, r.cy, r.Lp, r.Ln, r.ex, r.ey, r.ux, r.uy, r.tn, r.tp, r.opp_flags >> 1,
            (r.opp_flags & 1) != 0};
}

__device__ inline int lane_id() { return threadIdx.x; }
// Ends one step of a loop that applies the lanes' updates to a shared table
// one lane at a time: the next lane's loads must see this lane's stores. To
// the compiler the lanes are separate threads, so without this it may keep a
// table value in a register from one step to the next.
__device__ inline void lane_step_barrier() { __asm__ __volatile__("" ::: "memory"); }
__device__ inline uint64_t lanemask_lt() { return (1ull << threadIdx.x) - 1ull; }

__device__ inline double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

template <typename R>
__device__ inline R seg_dist(R px, R py, R b0, R b1) {
    R dx = px < b0 ? b0 - px : (px > b1 ? px - b1 : R(0));
    return sqrt(dx * dx + py * py);
}

// Parameters of the bend-vertex updates: 1 - re-launch tolerance, the
// angle under which two initial directions count as one, the tie band.
struct RootCfg {
    double keep, tie_dir, tie_rel;
};

// Bend-vertex (pseudo-source) table of one source, in a per-wavefront
// global area indexed by the mesh's bend-vertex number (pidx), so a source
// may reach any number of saddle and boundary vertices: rD the best distance
// so far, rL the distance of the last launch, (rtx, rty) the initial tangent
// of the best path, rD2 the best distance of a path leaving the source in
// another direction (the vertex's own tie gap, passed on to everything
// reached through it). queued marks a vertex on the pending-launch list
// pend; touched lists the vertices the source has reached, whose entries
// are reset when the source is done (a fresh entry has rD = rL = rD2 =
// infinity and queued = 0, so every source starts from an empty table
// without a sweep over the mesh); sel receives the vertices of a launch.
// An entry's fields form one 48-byte record (rD, rL, rtx, rty, rD2, queued),
// so that reading or updating it touches one or two cache lines rather than
// one per field; the three lists follow the records.
template <typename T>
struct RecField {
    char *base;  // field address of entry 0
    __device__ T &operator[](int64_t e) const { return *reinterpret_cast<T *>(base + e * kBendRec); }
};
struct BendTable {
    RecField<double> rD, rL, rtx, rty, rD2;
    RecField<int32_t> queued;
    int32_t *pend, *touched, *sel;
};

__device__ inline BendTable bend_table(char *base, int64_t stride, int slot, int rcap) {
    BendTable g;
    char *r = base + (int64_t)slot * stride;
    g.rD = {r};
    g.rL = {r + 8};
    g.rtx = {r + 16};
    g.rty = {r + 24};
    g.rD2 = {r + 32};
    g.queued = {r + 40};
    g.pend = reinterpret_cast<int32_t *>(r + (int64_t)rcap * kBendRec);
    g.touched = g.pend + rcap;
    g.sel = g.touched + rcap;
    return g;
}

// Wave-uniform state of the table and the LDS of one launch chunk.
struct BendLds {
    int32_t npend, ntouched;
    int32_t sface[8];  // the faces of the wavefront's sources (cutoff kernel)
    int32_t sel[kLaunchChunk];       // bend vertices of the chunk
    int32_t pref[kLaunchChunk + 1];  // prefix sums of their fan sizes
};

// Bend-vertex update (insert or improve): keep the smallest distance and
// its tangent, and the smallest distance of a path in another initial
// direction (directions closer than tie_dir count as one); `alt` is such a
// second distance that comes with the candidate (a path through another bend
// vertex carries that vertex's own second distance). Queue the vertex for a
// (re-)launch when its distance improved by more than the re-launch
// tolerance, when the direction of its best path changed, or when a path of
// another direction has just come within the tie band: everything already
// reached through the vertex then learns the new tangent or the tie.
// The lanes load their entries together and leave when their candidate
// cannot change anything (the stored distances only decrease); the others
// are applied one lane at a time in registers, each result passed to every
// lane holding the same vertex, and written back once.
// bend_update_loaded takes the entry loaded by the caller (bend_load,
// earlier, so that its latency overlaps other work; no other update of the
// table may come in between).
// Lane l's value of x (l wave-uniform): two scalar reads instead of a
// cross-lane permute.
__device__ inline double readlane_d(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
struct BendEntry {
    double D = INFINITY, D2 = INFINITY, L = INFINITY, tx = 0.0, ty = 0.0;
    int q = 1;
};
__device__ inline BendEntry bend_load(const BendTable &G, int e) {
    BendEntry c;
    c.D = G.rD[e];
    c.D2 = G.rD2[e];
    c.L = G.rL[e];
    c.tx = G.rtx[e];
    c.ty = G.rty[e];
    c.q = G.queued[e];
    return c;
}
__device__ inline void bend_update_loaded(const BendTable &G, BendLds &L, const RootCfg &rc, bool ok, int e, double d,
                                          double tx, double ty, double alt, const BendEntry &c) {
    double cD = c.D, cD2 = c.D2, cL = c.L, ax = c.tx, ay = c.ty;
    int qd = c.q;
    if (!ok) {
        cD = INFINITY;
        cD2 = INFINITY;
    } else if (d >= cD && d >= cD2 && alt >= cD2) {
        ok = false;
    }
    uint64_t m = __ballot(ok);
    if (!m) return;
    // list lengths, wave-uniform in registers
    int np = L.npend, nt = L.ntouched;
    // The usual case: every lane holds a different entry, so each update is
    // the lane's own, and they run at once (the lists are appended in lane
    // order, as one lane at a time would). Otherwise one lane at a time,
    // each result passed on to the lanes holding the same entry.
    bool dup = false;
    for (uint64_t r = m; r; r &= r - 1) {
        const int l = __ffsll((unsigned long long)r) - 1;
        dup |= ok && e == __builtin_amdgcn_readlane(e, l) && lane_id() != l;
    }
    if (!__ballot(dup)) {
        int app = 0, fresh = 0;
        if (ok) {
            fresh = !(cD < INFINITY);
            const bool differ = fabs(ax * ty - ay * tx) > rc.tie_dir || ax * tx + ay * ty < 0.0;
            const bool tied = cD2 - cD <= rc.tie_rel * cD;
            if (d < cD) {
                if (differ) {
                    cD2 = fmin(cD2, cD);
                    cL = INFINITY;
                }
                cD = d;
                ax = tx;
                ay = ty;
            } else if (differ) {
                cD2 = fmin(cD2, d);
            }
            cD2 = fmin(cD2, alt);
            if (!tied && cD2 - cD <= rc.tie_rel * cD) cL = INFINITY;
            if (cD < cL * rc.keep && !qd) {
                qd = 1;
                app = 1;
            }
        }
        const uint64_t ma = __ballot(app), mf = __ballot(fresh);
        if (app) G.pend[np + __popcll(ma & lanemask_lt())] = e;
        if (fresh) G.touched[nt + __popcll(mf & lanemask_lt())] = e;
        np += __popcll(ma);
        nt += __popcll(mf);
        m = 0;
    }
    while (m) {
        const int l = __ffsll((unsigned long long)m) - 1;
        int app = 0, fresh = 0;
        if (lane_id() == l) {
            // a fresh entry has cD = cL = cD2 = infinity: every branch below then inserts
            fresh = !(cD < INFINITY);
            const bool differ = fabs(ax * ty - ay * tx) > rc.tie_dir || ax * tx + ay * ty < 0.0;
            const bool tied = cD2 - cD <= rc.tie_rel * cD;
            if (d < cD) {
                if (differ) {
                    cD2 = fmin(cD2, cD);
                    cL = INFINITY;  // new direction: launch again however small the gain
                }
                cD = d;
                ax = tx;
                ay = ty;
            } else if (differ) {
                cD2 = fmin(cD2, d);
            }
            cD2 = fmin(cD2, alt);
            if (!tied && cD2 - cD <= rc.tie_rel * cD) cL = INFINITY;  // a new tie
            if (cD < cL * rc.keep && !qd) {
                qd = 1;
                app = 1;
                G.pend[np] = e;
            }
            if (fresh) G.touched[nt] = e;
        }
        np += __builtin_amdgcn_readlane(app, l);
        nt += __builtin_amdgcn_readlane(fresh, l);
        const int el = __builtin_amdgcn_readlane(e, l);
        const double bD = readlane_d(cD, l), bD2 = readlane_d(cD2, l), bL = readlane_d(cL, l);
        const double bx = readlane_d(ax, l), by = readlane_d(ay, l);
        const int bq = __builtin_amdgcn_readlane(qd, l);
        if (ok && e == el) {
            cD = bD;
            cD2 = bD2;
            cL = bL;
            ax = bx;
            ay = by;
            qd = bq;
        }
        m &= m - 1;
    }
    if (ok) {
        G.rD[e] = cD;
        G.rD2[e] = cD2;
        G.rL[e] = cL;
        G.rtx[e] = ax;
        G.rty[e] = ay;
        G.queued[e] = qd;
    }
    if (lane_id() == 0) {
        L.npend = np;
        L.ntouched = nt;
    }
    __syncthreads();  // later loads of the table, by any lane, see these values
}
__device__ inline void bend_update(const BendTable &G, BendLds &L, const RootCfg &rc, bool ok, int e, double d,
                                   double tx, double ty, double alt) {
    BendEntry c;
    if (ok) c = bend_load(G, e);
    bend_update_loaded(G, L, rc, ok, e, d, tx, ty, alt, c);
}

// A window of bend vertex w.root is stale when it comes from an earlier
// launch (its sg, rounded like every window of a launch, exceeds that of the
// last launch rL) or when the vertex has improved enough for a new launch.
template <typename R>
__device__ inline bool bend_stale(double rD, double rL, const Win<R> &w, const RootCfg &rc) {
    return w.sg > (R)rL || rD < rL * rc.keep;
}

// Empty the table again for the next source (only the entries it touched).
__device__ inline void bend_reset(const BendTable &G, BendLds &L) {
    const int nt = L.ntouched;
    for (int k = lane_id(); k < nt; k += kWave) {
        const int e = G.touched[k];
        G.rD[e] = INFINITY;
        G.rL[e] = INFINITY;
        G.rD2[e] = INFINITY;
        G.queued[e] = 0;
    }
    if (lane_id() == 0) {
        L.npend = 0;
        L.ntouched = 0;
    }
    __syncthreads();
}

// Two-level window stack: LDS first, a per-wave global area for overflow.
template <typename R>
struct Stack {
    using Rec = typename RecOf<R>::T;
    int kL;  // LDS records
    Rec *lds;
    Rec *glb;
    int gcap;
    int lsp, gsp;

    __device__ void push(bool want, const Win<R> &w, bool &overflow) {
        uint64_t m = __ballot(want);
        int cnt = __popcll(m);
        if (!cnt) return;
        int r = __popcll(m & lanemask_lt());
        int space = kL - lsp;
        if (want) {
            if (r < space) {
                store_rec(lds[lsp + r], w);
            } else {
                int pos = gsp + (r - space);
                if (pos < gcap) store_rec(glb[pos], w);
                else overflow = true;
            }
        }
        int to_l = min(cnt, space);
        lsp += to_l;
        gsp = min(gsp + (cnt - to_l), gcap);
    }
    // refill lanes without a window; returns whether any lane holds one
    __device__ bool refill(bool &have, Win<R> &w) {
        uint64_t need = __ballot(!have);
        int nneed = __popcll(need);
        int r = __popcll(need & lanemask_lt());
        int take_l = min(nneed, lsp);
        if (!have && r < take_l) {
            load_rec(lds[lsp - 1 - r], w);
            have = true;
        }
        lsp -= take_l;
        if (nneed > take_l && gsp > 0) {
            __syncthreads();  // make earlier global pushes of other lanes visible
            int take_g = min(nneed - take_l, gsp);
            if (!have && r >= take_l && r < take_l + take_g) {
                load_rec(glb[gsp - 1 - (r - take_l)], w);
                have = true;
            }
            gsp -= take_g;
        }
        return __ballot(have) != 0;
    }
};

// Child intervals. Left child: across C->A (stored on tp, frame origin A,
// x towards C). Right child: across B->C (stored on tn, frame origin C, x
// towards B). The endpoint intersections are evaluated in FP64 in both
// precisions.
template <typename R>
__device__ inline void child_left(const He<R> &h, const Win<R> &w, double txc, bool full, double &x0, double &x1) {
    if (full) {
        x0 = 0.0;
        x1 = (double)h.Lp;
        return;
    }
    const double px = w.px, py = w.py, b0 = w.b0, b1 = w.b1, cx = h.cx, cy = h.cy, Lp = h.Lp;
    x0 = b0 <= 0.0 ? 0.0 : Lp * (py * b0) / (py * cx + cy * (b0 - px));
    x1 = b1 >= txc ? Lp : Lp * (py * b1) / (py * cx + cy * (b1 - px));
    x0 = fmin(fmax(x0, 0.0), Lp);
    x1 = fmin(fmax(x1, 0.0), Lp);
}
template <typename R>
__device__ inline void child_right(const He<R> &h, const Win<R> &w, double txc, bool full, double &x0, double &x1) {
    if (full) {
        x0 = 0.0;
        x1 = (double)h.Ln;
        return;
    }
    const double px = w.px, py = w.py, b0 = w.b0, b1 = w.b1, cx = h.cx, cy = h.cy, L = h.L, Ln = h.Ln;
    x0 = b0 <= txc ? 0.0 : Ln * ((px - cx) * (-py) - (py - cy) * (b0 - px)) / ((L - cx) * (-py) + cy * (b0 - px));
    x1 = b1 >= L ? Ln : Ln * ((px - cx) * (-py) - (py - cy) * (b1 - px)) / ((L - cx) * (-py) + cy * (b1 - px));
    x0 = fmin(fmax(x0, 0.0), Ln);
    x1 = fmin(fmax(x1, 0.0), Ln);
}

// Frame changes into the child windows (the interval [x0, x1] already
// computed): left child on twin(prev(h)) with origin A, right child on
// twin(next(h)) with origin C.
template <typename R>
__device__ inline void make_left(const He<R> &h, const Win<R> &w, double x0, double x1, Win<R> &cl) {
    const R ex = h.ex, ey = h.ey;
    cl.px = ex * w.px + ey * w.py;
    cl.py = ex * w.py - ey * w.px;
    cl.b0 = (R)x0;
    cl.b1 = (R)x1;
    cl.sg = w.sg;
    cl.c = w.c * ex - w.s * ey;
    cl.s = w.s * ex + w.c * ey;
    cl.he = h.tp;
    cl.root = w.root;
}
template <typename R>
__device__ inline void make_right(const He<R> &h, const Win<R> &w, double x0, double x1, Win<R> &cr) {
    const R ux = h.ux, uy = h.uy;
    const R qx = w.px - h.cx, qy = w.py - h.cy;
    cr.px = ux * qx + uy * qy;
    cr.py = ux * qy - uy * qx;
    cr.b0 = (R)x0;
    cr.b1 = (R)x1;
    cr.sg = w.sg;
    cr.c = w.c * ux - w.s * uy;
    cr.s = w.s * ux + w.c * uy;
    cr.he = h.tn;
    cr.root = w.root;
}

__device__ inline void face_xyz(const DevMesh &m, int f, int k, double F3[3][3], double U3[3][3]) {
    const double *p = m.fpos + 18 * (int64_t)f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int q = (k + i) % 3;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            F3[i][d] = p[3 * q + d];
            U3[i][d] = p[9 + 3 * q + d];
        }
    }
}

}  // namespace wnd
}  // namespace gsim
