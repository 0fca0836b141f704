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
//
// Pruning (all exact for every pair closer than the cutoff):
//  - the paper's submeshing by the Euclidean lower bound (Sec. 3.1), done
//    implicitly: a window is dropped once sg + dist(p, interval) reaches the
//    cutoff;
//  - target-directed: any path through a window to target j has length at
//    least sg + dist(p, interval) + |X - x_j| for the 3D crossing point X on
//    the window's edge slice. A window is dropped when that bound reaches,
//    for every candidate target, the cutoff or the target's best distance so
//    far (widened by the tie gap so second-best directions are still seen).
//    A bend vertex reached only through dropped windows can only lead to
//    pairs that are beyond the cutoff or already matched.
//
// Bend vertices (pseudo-sources) are launched as a full fan of windows with
// sg = their distance, either as soon as they are found or improved (eager)
// or when no window is left (bucketed by `launch_delta`). Windows of a root
// whose distance improved after they were made are stale and dropped. The
// last launch of every bend vertex carries its final distance, so the
// processing order changes only the amount of work.
//
// Precision: FP64 throughout, or FP32 windows (half the register, stack and
// record bytes) with the child-interval endpoint intersections computed in
// FP64; a source with any pair within the guard band of the cutoff is then
// recomputed at once in FP64 by the same wavefront, so neighbour sets stay
// exact.
//
// Mapping to CDNA4: one wavefront per source (one workgroup per source when
// there are no more sources than resident slots, else a persistent grid that
// claims them, up to four neighbouring sources per wavefront; either way
// sources in spatial cell order from eight per-XCD chunks so each XCD's L2
// serves one region of the mesh); each lane holds one live window in
// registers; a lane with two children keeps one and pushes the other onto an
// LDS window stack (ballot/popcount compaction; a per-wave global overflow
// area takes what does not fit); idle lanes pop. The target table lives in
// LDS; the bend-vertex table is a per-wavefront table in global memory
// indexed by the mesh's bend-vertex number (any number of bend vertices per
// source), emptied through its touched list. Lanes updating different
// entries of either table do so at once, lanes on the same entry one at a
// time by a ballot loop (no atomics, deterministic in wave order). The LDS
// stack depth is a template parameter: a shallower stack lowers the
// workgroup's LDS footprint and lets more wavefronts share a compute unit.
//
// Batches: the sources of several surfaces (each with its own mesh, cutoff
// and particles) form one flattened index space served by the same grid; a
// wavefront finds its source's surface from the batch boundaries and reads
// that surface's descriptor. The grid's statistics go into one of several
// counter slots (by workgroup), so that they do not serialise on one line.
//
// Fused update (time steps with few sources, one workgroup per source): once
// the source's row is final, lane 0 applies the force sum over the row (Sec. 3.1),
// the integrator (Sec. 2.1) and the walk (Sec. 3.2) to that particle and
// writes its new state into next-state arrays, which no source reads during
// the pass; the row is read back with the same code as the separate update
// kernel, so the trajectory is bit-identical to it.
#include <hip/hip_ext.h>

#include <cmath>
#include <type_traits>

#include "gsim_internal.h"
#include "walk.h"
#include "window.h"

namespace gsim {
namespace {

using namespace wnd;

constexpr int kMaxCand = kCandCap;
constexpr int kHash = 256;
// Several sources per wavefront (kG of them, the grouped instantiations):
// each takes 1/kG of the target table and of the hash buckets.
constexpr int kMaxGroup = 8;
template <int kG>
constexpr int kGroupCand = kMaxCand / kG;
template <int kG>
constexpr int kGroupBuckets = kHash / kG;
constexpr int kBigStk = 8192;  // LDS window stack of the big-candidate instantiation
constexpr int kChunks = 8;
static_assert(kChunks == kWorkChunks, "one work counter per chunk");

struct GeoArgs {
    const SurfDesc *sd;  // [nsurf] surface descriptors
    BatchIdx bi;         // flattened source index -> surface
    GeoParams gp;
    void *stack;         // per wave: stack_cap records of 64 bytes
    int32_t *work;       // [kChunks] work counters
    Counters *ctr;
    int grab;            // consecutive sources claimed at a time
    char *roots;         // per wave: a bend-vertex table (rstride bytes, rcap vertices)
    int64_t rstride;
    int rcap;
    char *gtab;          // big-candidate mode: per wave the target arrays of gcap targets (gstride bytes)
    int64_t gstride;
    int gcap;
    int pre_cand;        // the candidate rows and counts were written ahead of the pass (k_candidates)
};

// The target table of one source: per candidate target its index, face,
// next target of the same face bucket, barycentrics, position with the
// current pruning bound, best and other-direction distances and the best
// tangent; a hash of faces to chains of targets; the bend-vertex state.
// Either all in LDS (at most kMaxCand targets, Lds), or, for sources with
// more candidates, the per-target arrays in a per-wavefront global area and
// the rest in LDS (GTab): the helpers below are written once for both.
struct Lds {
    static constexpr bool kBig = false;
    static constexpr int kBuckets = kHash;
    int32_t tj[kMaxCand], tface[kMaxCand], tnext[kMaxCand];
    double tb[kMaxCand][3];
    alignas(16) double cb[kMaxCand][4];  // target position and current pruning bound
    double d1[kMaxCand], d2[kMaxCand], t1x[kMaxCand], t1y[kMaxCand];
    int32_t head[kHash];
    int32_t ncand;
    int32_t ncg[kMaxGroup];  // candidate counts of the searches of a group's sources
    // the group being propagated (sources, rows, counts) and the sources that
    // wait to run alone: in LDS rather than in registers the propagation needs
    int32_t gsrc[kMaxGroup], gnc[kMaxGroup], galone[kMaxGroup];
    int32_t gall[kMaxGroup];  // the sources a group's search covers
    int64_t gc0[kMaxGroup];
    BendLds B;
};

// Big-candidate mode: hash heads, the bend-vertex state and the sort buffer
// of the candidate search in LDS.
constexpr int kBigHash = 1024;
constexpr int kBigSort = kBigCandMax;  // candidates are sorted in LDS
struct LdsBig {
    int32_t head[kBigHash];
    int32_t ncand;
    int32_t key[kBigSort];
    BendLds B;
};
struct GTab {
    static constexpr bool kBig = true;
    static constexpr int kBuckets = kBigHash;
    int32_t *tj, *tface, *tnext;
    double (*tb)[3];
    double (*cb)[4];
    double *d1, *d2, *t1x, *t1y;
    int32_t *head;
    int32_t &ncand;
    BendLds &B;
};
// Bytes of one wavefront's global target arrays for gcap targets.
__host__ __device__ inline int64_t gtab_bytes(int gcap) { return ((int64_t)gcap * 100 + 255) / 256 * 256; }
__device__ inline GTab gtab_of(char *base, int64_t stride, int slot, int gcap, LdsBig &LB) {
    char *p = base + (int64_t)slot * stride;
    double *dp = reinterpret_cast<double *>(p);  // the doubles first: 11 per target
    double(*cb)[4] = reinterpret_cast<double(*)[4]>(dp);
    double(*tb)[3] = reinterpret_cast<double(*)[3]>(dp + 4 * (int64_t)gcap);
    double *d1 = dp + 7 * (int64_t)gcap;
    int32_t *ip = reinterpret_cast<int32_t *>(dp + 11 * (int64_t)gcap);
    return GTab{ip, ip + gcap, ip + 2 * (int64_t)gcap, tb, cb, d1, d1 + gcap, d1 + 2 * (int64_t)gcap,
                d1 + 3 * (int64_t)gcap, LB.head, LB.ncand, LB.B};
}

// Multiplicative hash of a face index: the top bits of f times the golden
// ratio in 32-bit fixed point (256 buckets: the top 8 bits). kB buckets per
// source: the table's own count, or half of it for each source of a pair.
template <int kB>
__device__ inline int hash_bits(int f) {
    static_assert(kB == 32 || kB == 64 || kB == 128 || kB == 256 || kB == 1024, "bucket counts");
    constexpr int kShift = kB == 32 ? 27 : (kB == 64 ? 26 : (kB == 128 ? 25 : (kB == 256 ? 24 : 22)));
    return (int)(((uint32_t)f * 2654435761u) >> kShift) & (kB - 1);
}
template <class TL>
__device__ inline int hash_face(int f) {
    return hash_bits<TL::kBuckets>(f);
}

// First target of face f in the table of the source whose buckets start at
// hb (kB of them).
template <class TL, int kB = TL::kBuckets>
__device__ inline int first_in_face(const TL &L, int f, int hb = 0) {
    int s = L.head[hb + hash_bits<kB>(f)];
    while (s >= 0 && L.tface[s] != f) s = L.tnext[s];
    return s;
}
template <class TL>
__device__ inline int next_in_face(const TL &L, int s, int f) {
    s = L.tnext[s];
    while (s >= 0 && L.tface[s] != f) s = L.tnext[s];
    return s;
}

// The wavefront's sources: one, or in the grouped instantiations (kG = 2 or
// 4) up to kG of the same surface, sharing the lanes, the window stack and
// the bend-vertex table. Source q of a group owns targets [q kGroupCand,
// ...) and hash buckets [q kGroupBuckets, ...) of the table, and entry
// kG v + q of bend vertex v (a group's sources are neighbours and reach
// mostly the same bend vertices: interleaved, their entries share cache
// lines); its source windows carry root -1 - q, its bend-vertex windows the
// entry index, so every window knows its source. A lone source of a grouped
// instantiation takes the whole table.
template <int kG>
__device__ inline int slot_of(int root) {
    static_assert(kG == 1 || kG == 2 || kG == 4 || kG == 8, "group sizes");
    if constexpr (kG == 1) {
        return 0;
    } else {
        return root >= 0 ? root & (kG - 1) : -1 - root;
    }
}
// bend-vertex entry of vertex number v (pidx) for source q, and back
template <int kG>
__device__ inline int bend_entry(int v, int q) {
    return kG == 1 ? v : v * kG + q;
}
template <int kG>
__device__ inline int bend_vertex(int e) {
    return kG == 1 ? e : e / kG;
}

// Per-source constants shared by the helpers.
struct Ctx {
    double cutoff, cut_acc, lb_slack, tol, tie_rel, tie_dir;
    double root_keep;  // 1 - relative improvement below which a bend vertex is not re-launched
    RootCfg rc;
    int nc;
    int nc4;  // nc rounded up to a multiple of 4 (the padded bound table)
};

// Could a path of length `base` to the edge slice P + x u (x in [x0, x1])
// still improve some candidate target? (3D distance as the lower bound of
// the rest of the path.) Targets are tested four at a time, so that their
// independent load and arithmetic chains overlap; the bound table is padded
// to a multiple of four with entries that no path can reach.
template <class TL>
__device__ inline bool reaches_target(const TL &L, const Ctx &C, const double P[3], const double u[3], double x0,
                                      double x1, double base, int tb = 0, int nc4 = -1) {
    // with more targets than the LDS table holds, nearly every window within
    // the cutoff can still improve one of them: only the cutoff prunes
    if constexpr (TL::kBig) return base < C.cut_acc;
    const int te = tb + (nc4 < 0 ? C.nc4 : nc4);  // the source's targets: [tb, te)
    for (int s0 = tb; s0 < te; s0 += 4) {
        bool hit = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double *cb = L.cb[s0 + i];
            const double rem = cb[3] - base;
            double q0 = cb[0] - P[0], q1 = cb[1] - P[1], q2 = cb[2] - P[2];
            double t = q0 * u[0] + q1 * u[1] + q2 * u[2];
            t = fmin(fmax(t, x0), x1);
            q0 -= t * u[0];
            q1 -= t * u[1];
            q2 -= t * u[2];
            hit |= rem > 0.0 && q0 * q0 + q1 * q1 + q2 * q2 < rem * rem;
        }
        if (hit) return true;
    }
    return false;
}

// Target update: best distance, its tangent, and the best
// distance among candidates whose direction differs (tie gap); `alt` is the
// distance of another-direction path that comes with the candidate (through
// a bend vertex with a second distance).
template <class TL>
__device__ inline void target_update(TL &L, const Ctx &C, bool ok, int slot, double d, double tx, double ty,
                                     double alt) {
    // candidates no shorter than both distances (which only decrease) change nothing
    if (ok && d >= L.d1[slot] && d >= L.d2[slot] && alt >= L.d2[slot]) ok = false;
    uint64_t m = __ballot(ok);
    if (!m) return;
    // lanes on different targets (the usual case) update at once, else one
    // lane at a time
    bool dup = false;
    for (uint64_t r = m; r; r &= r - 1) {
        const int l = __ffsll((unsigned long long)r) - 1;
        dup |= ok && slot == __builtin_amdgcn_readlane(slot, l) && lane_id() != l;
    }
    if (!__ballot(dup)) m = 0;
    if (!m && ok) {
        double c1 = L.d1[slot];
        double ax = L.t1x[slot], ay = L.t1y[slot];
        bool differ = !(c1 < INFINITY) || fabs(ax * ty - ay * tx) > C.tie_dir || ax * tx + ay * ty < 0.0;
        if (d < c1) {
            if (differ) L.d2[slot] = fmin(L.d2[slot], c1);
            L.d1[slot] = d;
            L.t1x[slot] = tx;
            L.t1y[slot] = ty;
            L.cb[slot][3] = fmin(C.cut_acc, d * (1.0 + C.tie_rel) + C.lb_slack);
        } else if (differ) {
            L.d2[slot] = fmin(L.d2[slot], d);
        }
        L.d2[slot] = fmin(L.d2[slot], alt);
    }
    lane_step_barrier();
    while (m) {
        int l = __ffsll((unsigned long long)m) - 1;
        if (lane_id() == l) {
            double c1 = L.d1[slot];
            double ax = L.t1x[slot], ay = L.t1y[slot];
            bool differ = !(c1 < INFINITY) || fabs(ax * ty - ay * tx) > C.tie_dir || ax * tx + ay * ty < 0.0;
            if (d < c1) {
                if (differ) L.d2[slot] = fmin(L.d2[slot], c1);
                L.d1[slot] = d;
                L.t1x[slot] = tx;
                L.t1y[slot] = ty;
                L.cb[slot][3] = fmin(C.cut_acc, d * (1.0 + C.tie_rel) + C.lb_slack);
            } else if (differ) {
                L.d2[slot] = fmin(L.d2[slot], d);
            }
            L.d2[slot] = fmin(L.d2[slot], alt);
        }
        lane_step_barrier();
        m &= m - 1;
    }
}

// Both children of a window. F3: the face's vertices in 3D in the order
// (A, B, C) = (tail, head, opposite) of the entry half-edge; U3: the unit
// directions of the half-edges (A->B, B->C, C->A).
template <typename R, class TL>
__device__ inline void children(const He<R> &h, const Win<R> &w, double txc, bool full, const Ctx &C,
                                const double F3[3][3], const double U3[3][3], const TL &L, Win<R> &cl, bool &hl,
                                Win<R> &cr, bool &hr, int &pruned, int tb = 0, int nc4 = -1) {
    hl = false;
    hr = false;
    if (h.tp >= 0 && (full || (double)w.b0 < txc)) {
        double x0, x1;
        child_left(h, w, txc, full, x0, x1);
        make_left(h, w, x0, x1, cl);
        if (x1 - x0 > 1e-12 * (double)h.Lp) {
            const double base = (double)w.sg + (double)seg_dist(cl.px, cl.py, cl.b0, cl.b1);
            // edge A -> C is the reverse of half-edge prev = (C -> A)
            const double u[3] = {-U3[2][0], -U3[2][1], -U3[2][2]};
            if (reaches_target(L, C, F3[0], u, x0, x1, base, tb, nc4)) hl = true;
            else ++pruned;
        }
    }
    if (h.tn >= 0 && (full || (double)w.b1 > txc)) {
        double x0, x1;
        child_right(h, w, txc, full, x0, x1);
        make_right(h, w, x0, x1, cr);
        if (x1 - x0 > 1e-12 * (double)h.Ln) {
            const double base = (double)w.sg + (double)seg_dist(cr.px, cr.py, cr.b0, cr.b1);
            // edge C -> B is the reverse of half-edge next = (B -> C)
            const double u[3] = {-U3[1][0], -U3[1][1], -U3[1][2]};
            if (reaches_target(L, C, F3[2], u, x0, x1, base, tb, nc4)) hr = true;
            else ++pruned;
        }
    }
}

struct SrcStats {
    unsigned long long windows, launches, stale, guards;
    int pruned;
    int depth;  // deepest window stack (records)
    bool overflow;
};

// Launch the pending bend vertices (distance improved since their last
// launch, direction changed or a tie appeared) within launch_delta of the
// smallest such distance; the others stay pending. The selected vertices
// are compacted into a list and their fans flattened over the lanes, a chunk
// of vertices at a time, so one launch round costs a few memory round trips,
// not one per vertex. In the grouped instantiations entry e stands for bend
// vertex e / kG of source e mod kG (its targets from q tspan on).
template <typename R, class TL, int kG = 1>
__device__ void launch_roots(const GeoArgs &a, const SurfDesc &sd, TL &L, const BendTable &G, const Ctx &C,
                             Stack<R> &S, SrcStats &st, int tspan = 0, const int *ncs = nullptr) {
    constexpr int kB = kG == 1 ? TL::kBuckets : kGroupBuckets<kG>;
    const int lane = lane_id();
    const DevMesh &M = sd.m;
    const HeRec *__restrict__ he = M.he;
    const int npend = L.B.npend;
    // the first wavefront's worth of pending entries is read once for both
    // passes below
    int e0 = 0;
    double D0 = 0.0, L0 = INFINITY;
    if (lane < npend) {
        e0 = G.pend[lane];
        D0 = G.rD[e0];
        L0 = G.rL[e0];
    }
    double mn = INFINITY;
    for (int k = lane; k < npend; k += kWave) {
        double D = D0, Lr = L0;
        if (k >= kWave) {
            const int e = G.pend[k];
            D = G.rD[e];
            Lr = G.rL[e];
        }
        if (D < Lr * C.rc.keep && D < C.cut_acc) mn = fmin(mn, D);
    }
    mn = wave_min(mn);
    const double thr = mn + a.gp.launch_delta;
    // 1. split the pending list: launch now (marked launched), keep pending
    //    (compacted in place: a kept entry never moves past its own slot), or
    //    drop (nothing left to launch)
    int nsel = 0, nkeep = 0;
    for (int base = 0; base < npend; base += kWave) {
        const int k = base + lane;
        int e = 0;
        bool sel = false, keep = false;
        double D = 0.0;
        if (k < npend) {
            double Lr = L0;
            if (base == 0) {
                e = e0;
                D = D0;
            } else {
                e = G.pend[k];
                D = G.rD[e];
                Lr = G.rL[e];
            }
            const bool cand = D < Lr * C.rc.keep && D < C.cut_acc;
            sel = cand && D <= thr;
            keep = cand && !sel;
        }
        const uint64_t ms = __ballot(sel), mk = __ballot(keep);
        if (sel) {
            const int pos = nsel + __popcll(ms & lanemask_lt());
            G.sel[pos] = e;
            if (pos < kLaunchChunk) L.B.sel[pos] = e;  // the first chunk also through LDS
            G.rL[e] = D;
        }
        if (keep) G.pend[nkeep + __popcll(mk & lanemask_lt())] = e;
        if (k < npend && !keep) G.queued[e] = 0;
        nsel += __popcll(ms);
        nkeep += __popcll(mk);
    }
    if (lane == 0) L.B.npend = nkeep;
    __syncthreads();
    for (int c0 = 0; c0 < nsel; c0 += kLaunchChunk) {
        const int cn = min(kLaunchChunk, nsel - c0);
        // 2. per vertex: is any target within reach (3D bound), and its fan size
        int carry = 0;
        for (int base = 0; base < cn; base += kWave) {
            const int k = base + lane;
            int deg = 0;
            if (k < cn) {
                int e;
                if (c0 == 0) {
                    e = L.B.sel[k];
                } else {
                    e = G.sel[c0 + k];
                    L.B.sel[k] = e;
                }
                const int q = slot_of<kG>(e);
                const PseudoRec pr = M.prec[bend_vertex<kG>(e)];
                const double D = G.rD[e];
                // big-candidate mode: every vertex within the cutoff (as for windows)
                bool useful = TL::kBig;
                const int tb = q * tspan, te = tb + (kG == 1 ? C.nc : ncs[q]);
                for (int s = tb; !TL::kBig && s < te && !useful; ++s) {
                    const double bound = L.cb[s][3] - D;
                    const double q0 = L.cb[s][0] - pr.x, q1 = L.cb[s][1] - pr.y, q2 = L.cb[s][2] - pr.z;
                    useful = bound > 0.0 && q0 * q0 + q1 * q1 + q2 * q2 < bound * bound;
                }
                if (useful) deg = pr.fan_deg;
            }
            // wave-inclusive scan of deg
            int inc = deg;
            for (int o = 1; o < kWave; o <<= 1) {
                const int y = __shfl_up(inc, o);
                if (lane >= o) inc += y;
            }
            if (k < cn) L.B.pref[k + 1] = carry + inc;
            st.launches += (unsigned long long)__popcll(__ballot(deg > 0));
            carry += __builtin_amdgcn_readlane(inc, kWave - 1);
        }
        if (lane == 0) L.B.pref[0] = 0;
        __syncthreads();
        const int total = carry;
        // 3. flattened fans: lane <- (vertex k, fan position)
        for (int base = 0; base < total; base += kWave) {
            const int idx = base + lane;
            const bool act = idx < total;
            int k = 0;
            if (act) {
                int lo = 0, hi = cn - 1;  // largest k with pref[k] <= idx
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (L.B.pref[mid] <= idx) lo = mid;
                    else hi = mid - 1;
                }
                k = lo;
            }
            const int el = act ? L.B.sel[k] : 0;
            const int q = slot_of<kG>(el);  // the vertex's source
            const int tb = q * tspan, hb = q * kB;
            PseudoRec pr{0.0, 0.0, 0.0, 0, 0, 0, 0};
            if (act) pr = M.prec[bend_vertex<kG>(el)];
            const double D = act ? G.rD[el] : 0.0;
            const double vtx = act ? G.rtx[el] : 0.0, vty = act ? G.rty[el] : 0.0;
            const double D2 = act ? G.rD2[el] : INFINITY;  // the vertex's other-direction distance
            const int h = act ? M.fan[pr.fan_beg + (idx - L.B.pref[k])] : 0;
            const int hn = h - h % 3 + (h % 3 + 1) % 3;
            const HeRec Rh = he[h], Rn = he[hn];
            Win<R> nw;
            bool want = false;
            if (act && Rn.twin >= 0) {
                // window across the edge opposite v: twin(next(h)) runs u2 -> u1
                const double px = Rn.L - Rn.cx, py = -Rn.cy;
                nw.px = (R)px;
                nw.py = (R)py;
                nw.b0 = R(0);
                nw.b1 = (R)Rn.L;
                nw.sg = (R)D;
                nw.c = R(1);
                nw.s = R(0);
                nw.he = Rn.twin;
                nw.root = el;
                double F3[3][3], U3[3][3];
                face_xyz(M, h / 3, h % 3, F3, U3);  // (v, u1, u2)
                // the window's edge runs u2 -> u1: the reverse of half-edge next(h) = (u1 -> u2)
                const double u[3] = {-U3[1][0], -U3[1][1], -U3[1][2]};
                want = reaches_target(L, C, F3[2], u, 0.0, Rn.L, D + seg_dist(px, py, 0.0, Rn.L), tb,
                                      kG == 1 ? C.nc4 : (ncs[q] + 3) & ~3);
            }
            // direct targets in face(h)
            const int g = h / 3;
            int slot = act ? first_in_face<TL, kB>(L, g, hb) : -1;
            while (__ballot(slot >= 0)) {
                const bool ok = slot >= 0;
                double d = 0;
                if (ok) {
                    const double dx = L.cb[slot][0] - pr.x, dy = L.cb[slot][1] - pr.y, dz = L.cb[slot][2] - pr.z;
                    d = D + sqrt(dx * dx + dy * dy + dz * dz);
                }
                target_update(L, C, ok, slot, d, vtx, vty, D2 + (d - D));
                if (ok) slot = next_in_face(L, slot, g);
            }
            // adjacent bend vertices along the two edges at v
            const int u1 = act ? Rh.head : 0;  // head of h
            const int p1 = act && D + Rh.L < C.cut_acc ? M.pidx[u1] : -1;
            bend_update(G, L.B, C.rc, p1 >= 0, bend_entry<kG>(p1, q), D + Rh.L, vtx, vty, D2 + Rh.L);
            const int u2 = act ? Rh.opp_flags >> 1 : 0;
            const int p2 = act && D + Rh.Lp < C.cut_acc ? M.pidx[u2] : -1;
            bend_update(G, L.B, C.rc, p2 >= 0, bend_entry<kG>(p2, q), D + Rh.Lp, vtx, vty, D2 + Rh.Lp);
            S.push(want, nw, st.overflow);
        }
        __syncthreads();  // the chunk arrays are rewritten by the next chunk
    }
}

// The group lists from a group search's counts (L.ncg, L.gall): sources
// with 1 .. kGroupCand candidates in order (gsrc, gc0, gnc; nb of them) and
// those with more (galone; na).
template <int kG, class LT>
__device__ void group_lists(LT &L, int ng, int &nb, int &na) {
    constexpr int kCap = kGroupCand<kG>;
    const int lane = lane_id();
    nb = na = 0;
    for (int q = 0; q < ng; ++q) {
        const int n = L.ncg[q];
        const int src = L.gall[q];
        if (n > kCap) {
            if (lane == 0) L.galone[na] = src;
            ++na;
        } else if (n > 0) {
            if (lane == 0) {
                L.gsrc[nb] = src;
                L.gc0[nb] = (int64_t)src * kMaxCand;
                L.gnc[nb] = n;
            }
            ++nb;
        }
    }
    __syncthreads();
}

// The LDS of the candidate-search kernel: the search's scratch and group
// lists only.
struct CandLds {
    int32_t tj[kMaxCand], tnext[kMaxCand];
    int32_t ncand;
    int32_t ncg[kMaxGroup], gsrc[kMaxGroup], gnc[kMaxGroup], galone[kMaxGroup], gall[kMaxGroup];
    int64_t gc0[kMaxGroup];
};

// Euclidean prefilter of one source (the lower bound of Sec. 3.1): lanes 0-26
// scan the 27 cells around it, the hits are rank-sorted by particle index in
// LDS and written out as the source's candidate row. Returns the true count
// (more than kMaxCand is an overflow the caller reports).
template <class LT>
__device__ int find_candidates(const SurfDesc &sd, LT &L, int src, int64_t c0) {
    constexpr int tb = 0, cap = kMaxCand;
    const int lane = lane_id();
    int32_t &ncand = L.ncand;
    if (lane == 0) ncand = 0;
    __syncthreads();
    const double xi = sd.xyz[3 * (int64_t)src], yi = sd.xyz[3 * (int64_t)src + 1], zi = sd.xyz[3 * (int64_t)src + 2];
    const int lin = sd.cell_of[src];
    const int cx = lin % sd.dims[0], cy = (lin / sd.dims[0]) % sd.dims[1], cz = lin / (sd.dims[0] * sd.dims[1]);
    if (lane < 27) {
        const int x = cx + lane % 3 - 1, y = cy + (lane / 3) % 3 - 1, z = cz + lane / 9 - 1;
        if (x >= 0 && x < sd.dims[0] && y >= 0 && y < sd.dims[1] && z >= 0 && z < sd.dims[2]) {
            const int c = (z * sd.dims[1] + y) * sd.dims[0] + x;
            const int e1 = sd.cell_start[c + 1];
            for (int q = sd.cell_start[c]; q < e1; ++q) {
                const int j = sd.order[q];
                if (j == src) continue;
                const double ex = sd.xyz[3 * (int64_t)j] - xi, ey = sd.xyz[3 * (int64_t)j + 1] - yi,
                             ez = sd.xyz[3 * (int64_t)j + 2] - zi;
                if (ex * ex + ey * ey + ez * ez < sd.cut2) {
                    const int pos = atomicAdd(&ncand, 1);
                    if (pos < cap) L.tnext[tb + pos] = j;
                }
            }
        }
    }
    __syncthreads();
    const int total = ncand;
    const int m = min(total, cap);
    for (int s = lane; s < m; s += kWave) {
        const int j = L.tnext[tb + s];
        int rank = 0;
        for (int t = 0; t < m; ++t) rank += L.tnext[tb + t] < j;
        L.tj[tb + rank] = j;
    }
    __syncthreads();
    for (int s = lane; s < m; s += kWave) sd.cand[c0 + s] = L.tj[tb + s];
    if (lane == 0) sd.cand_cnt[src] = total;
    return total;
}

// The Euclidean prefilter of a group's ng (at most kG) sources at once:
// those at positions p0 .. p0 + ng - 1 of the surface's cell order. Lane
// pairs (source, neighbour cell) scan the cells, two per lane, with their
// loads interleaved; source q's hits go to region q of kGroupCand entries,
// and are rank-sorted by particle index into the region of its place among
// the sources with 1 .. kGroupCand candidates (the group, in order: gsrc,
// gc0, gnc, nb of them), whose candidate rows are written. Sources with more
// go to galone (na of them) and are searched again alone; every count goes
// to cand_cnt. The same group and rows as searching the sources one by one.
template <int kG, class LT>
__device__ void find_candidates_group(const SurfDesc &sd, LT &L, int p0, int ng, int &nb, int &na) {
    constexpr int kCap = kGroupCand<kG>;
    const int lane = lane_id();
    if (lane < kG) L.ncg[lane] = 0;
    __syncthreads();
    constexpr int kPairs = (27 * kG + kWave - 1) / kWave;  // (source, cell) pairs per lane
    int beg[kPairs], len[kPairs], own[kPairs], qh[kPairs];
    double x[kPairs], y[kPairs], z[kPairs];
#pragma unroll
    for (int hh = 0; hh < kPairs; ++hh) {
        const int pr = lane + kWave * hh, q = pr / 27, l = pr - 27 * q;
        beg[hh] = len[hh] = 0;
        own[hh] = -1;
        qh[hh] = q;
        x[hh] = y[hh] = z[hh] = 0.0;
        if (q < ng) {
            const int src = sd.order[p0 + q];
            own[hh] = src;
            if (l == 0) L.gall[q] = src;
            x[hh] = sd.xyz[3 * (int64_t)src];
            y[hh] = sd.xyz[3 * (int64_t)src + 1];
            z[hh] = sd.xyz[3 * (int64_t)src + 2];
            const int lin = sd.cell_of[src];
            const int cx = lin % sd.dims[0] + l % 3 - 1, cy = (lin / sd.dims[0]) % sd.dims[1] + (l / 3) % 3 - 1,
                      cz = lin / (sd.dims[0] * sd.dims[1]) + l / 9 - 1;
            if (cx >= 0 && cx < sd.dims[0] && cy >= 0 && cy < sd.dims[1] && cz >= 0 && cz < sd.dims[2]) {
                const int c = (cz * sd.dims[1] + cy) * sd.dims[0] + cx;
                beg[hh] = sd.cell_start[c];
                len[hh] = sd.cell_start[c + 1] - beg[hh];
            }
        }
    }
    // four particles of each pair a step: their indices, then their
    // positions, each as one round of loads
    constexpr int kU = 4;
    const double cut2 = sd.cut2;
    int maxlen = 0;
#pragma unroll
    for (int hh = 0; hh < kPairs; ++hh) maxlen = max(maxlen, len[hh]);
    for (int it = 0; it < maxlen; it += kU) {
        int jj[kPairs][kU];
#pragma unroll
        for (int hh = 0; hh < kPairs; ++hh)
#pragma unroll
            for (int u = 0; u < kU; ++u) jj[hh][u] = it + u < len[hh] ? sd.order[beg[hh] + it + u] : -1;
        double dd[kPairs][kU];
#pragma unroll
        for (int hh = 0; hh < kPairs; ++hh)
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int j = jj[hh][u];
                dd[hh][u] = INFINITY;
                if (j >= 0 && j != own[hh]) {
                    const double ex = sd.xyz[3 * (int64_t)j] - x[hh], ey = sd.xyz[3 * (int64_t)j + 1] - y[hh],
                                 ez = sd.xyz[3 * (int64_t)j + 2] - z[hh];
                    dd[hh][u] = ex * ex + ey * ey + ez * ez;
                }
            }
#pragma unroll
        for (int hh = 0; hh < kPairs; ++hh)
#pragma unroll
            for (int u = 0; u < kU; ++u)
                if (dd[hh][u] < cut2) {
                    const int pos = atomicAdd(&L.ncg[qh[hh]], 1);
                    if (pos < kCap) L.tnext[qh[hh] * kCap + pos] = jj[hh][u];
                }
    }
    __syncthreads();
    // places: source q's index among the accepted ones (wave-uniform counts)
    auto place_of = [&](int q) {
        int pl = 0;
        for (int t = 0; t < q; ++t) pl += L.ncg[t] > 0 && L.ncg[t] <= kCap;
        return pl;
    };
    // ranks within each source's hits, which sit in kCap consecutive lanes of
    // a pass: compared through lane reads (absent entries hold INT_MAX)
    static_assert(kCap == 16 || kCap == 32 || kCap == 64, "one, two or four sources per pass");
    for (int base = 0; base < ng * kCap; base += kWave) {
        const int k = base + lane, q = k / kCap, s = k - q * kCap;
        const int m = q < ng ? L.ncg[q] : 0;
        const bool mine = m <= kCap && s < m;
        const int j = mine ? L.tnext[q * kCap + s] : INT_MAX;
        int rank = 0;
        for (int t = 0; t < kCap; ++t) {
            int v = __builtin_amdgcn_readlane(j, t);
#pragma unroll
            for (int b = 1; b < kWave / kCap; ++b)
                if (lane >= b * kCap) v = __builtin_amdgcn_readlane(j, b * kCap + t);
            rank += v < j;
        }
        if (mine) L.tj[place_of(q) * kCap + rank] = j;
    }
    __syncthreads();
    for (int k = lane; k < ng * kCap; k += kWave) {
        const int q = k / kCap, s = k - q * kCap, m = L.ncg[q];
        if (m <= kCap && s < m) sd.cand[(int64_t)L.gall[q] * kMaxCand + s] = L.tj[place_of(q) * kCap + s];
    }
    if (lane < ng) sd.cand_cnt[L.gall[lane]] = L.ncg[lane];
    group_lists<kG>(L, ng, nb, na);
}

// A group's sources from their candidate rows written ahead of the pass
// (k_candidates): counts, the rows of those with 1 .. kGroupCand candidates
// into their places' regions of the table, and the group lists.
template <int kG>
__device__ void take_candidates(const SurfDesc &sd, Lds &L, int p0, int ng, int &nb, int &na) {
    constexpr int kCap = kGroupCand<kG>;
    const int lane = lane_id();
    if (lane < ng) {
        const int src = sd.order[p0 + lane];
        L.gall[lane] = src;
        L.ncg[lane] = sd.cand_cnt[src];
    }
    __syncthreads();
    for (int k = lane; k < ng * kCap; k += kWave) {
        const int q = k / kCap, s = k - q * kCap, m = L.ncg[q];
        if (m <= kCap && s < m) {
            int pl = 0;
            for (int t = 0; t < q; ++t) pl += L.ncg[t] > 0 && L.ncg[t] <= kCap;
            L.tj[pl * kCap + s] = sd.cand[(int64_t)L.gall[q] * kMaxCand + s];
        }
    }
    group_lists<kG>(L, ng, nb, na);
}

// One source's candidate row written ahead of the pass into the table
// (as find_candidates leaves it); returns its count.
__device__ int take_row(const SurfDesc &sd, Lds &L, int src, int64_t c0) {
    const int n = sd.cand_cnt[src];
    for (int s = lane_id(); s < min(n, kMaxCand); s += kWave) L.tj[s] = sd.cand[c0 + s];
    __syncthreads();
    return n;
}

// The Euclidean prefilter of every source ahead of a grouped pass: kG
// consecutive sources of the cell order per wavefront (on one surface at a
// time), the same rows and counts as the search inside the pass, at the
// occupancy of a kernel with small LDS and register needs rather than that
// of the propagation.
template <int kG>
__global__ __launch_bounds__(kWave) void k_candidates(const SurfDesc *__restrict__ desc, BatchIdx bi) {
    __shared__ CandLds L;
    const int total = bi.begin[bi.nsurf];
    int pos = (int)blockIdx.x * kG;
    const int end = min(pos + kG, total);
    while (pos < end) {
        const int si = __builtin_amdgcn_readfirstlane(batch_surface(bi, pos));
        const SurfDesc &sd = desc[si];
        const int ng = min(end, bi.begin[si + 1]) - pos;
        int nb, na;
        find_candidates_group<kG>(sd, L, pos - bi.begin[si], ng, nb, na);
        for (int g = 0; g < na; ++g) {
            const int s1 = L.galone[g];
            find_candidates(sd, L, s1, (int64_t)s1 * kMaxCand);
        }
        pos += ng;
    }
}

// The Euclidean prefilter of one source in big-candidate mode: the 27 cells'
// particle ranges are flattened over the lanes, the hits collected in LDS,
// bitonic-sorted by particle index and written to the table and the row.
// Returns the true count (more than cap is an overflow the caller reports).
__device__ int find_candidates_big(const SurfDesc &sd, LdsBig &LB, GTab &T, int src, int64_t c0, int cap) {
    const int lane = lane_id();
    if (lane == 0) LB.ncand = 0;
    const double xi = sd.xyz[3 * (int64_t)src], yi = sd.xyz[3 * (int64_t)src + 1], zi = sd.xyz[3 * (int64_t)src + 2];
    const int lin = sd.cell_of[src];
    const int cx = lin % sd.dims[0], cy = (lin / sd.dims[0]) % sd.dims[1], cz = lin / (sd.dims[0] * sd.dims[1]);
    // lane l < 27: the particle range of neighbour cell l
    int b = 0, e = 0;
    if (lane < 27) {
        const int x = cx + lane % 3 - 1, y = cy + (lane / 3) % 3 - 1, z = cz + lane / 9 - 1;
        if (x >= 0 && x < sd.dims[0] && y >= 0 && y < sd.dims[1] && z >= 0 && z < sd.dims[2]) {
            const int c = (z * sd.dims[1] + y) * sd.dims[0] + x;
            b = sd.cell_start[c];
            e = sd.cell_start[c + 1];
        }
    }
    int inc = e - b;
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    const int total_in = __builtin_amdgcn_readlane(inc, 26);
    const int excl = inc - (e - b);
    // every cell's start in the flattened order and in the particle order, wave-uniform
    int cs[27], cb0[27];
#pragma unroll
    for (int l = 0; l < 27; ++l) {
        cs[l] = __builtin_amdgcn_readlane(excl, l);
        cb0[l] = __builtin_amdgcn_readlane(b, l);
    }
    __syncthreads();
    for (int q0 = 0; q0 < total_in; q0 += kWave) {
        const int q = q0 + lane;
        if (q >= total_in) continue;
        // the cell holding flattened position q: the last one starting at or before q
        int cell = 0;
#pragma unroll
        for (int l = 1; l < 27; ++l) cell = cs[l] <= q ? l : cell;
        int base = cb0[0], st0 = cs[0];
#pragma unroll
        for (int l = 1; l < 27; ++l)
            if (cell == l) {
                base = cb0[l];
                st0 = cs[l];
            }
        const int j = sd.order[base + (q - st0)];
        if (j == src) continue;
        const double ex = sd.xyz[3 * (int64_t)j] - xi, ey = sd.xyz[3 * (int64_t)j + 1] - yi,
                     ez = sd.xyz[3 * (int64_t)j + 2] - zi;
        if (ex * ex + ey * ey + ez * ez < sd.cut2) {
            const int pos = atomicAdd(&LB.ncand, 1);
            if (pos < kBigSort) LB.key[pos] = j;
        }
    }
    __syncthreads();
    const int total = LB.ncand;
    const int m = min(total, min(cap, kBigSort));
    int P = 1;
    while (P < m) P <<= 1;
    for (int s = m + lane; s < P; s += kWave) LB.key[s] = 0x7fffffff;
    __syncthreads();
    // bitonic sort of key[0, P) ascending
    for (int k = 2; k <= P; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int s = lane; s < P; s += kWave) {
                const int t = s ^ jj;
                if (t > s) {
                    const int a0 = LB.key[s], a1 = LB.key[t];
                    const bool up = (s & k) == 0;
                    if ((a0 > a1) == up) {
                        LB.key[s] = a1;
                        LB.key[t] = a0;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int s = lane; s < m; s += kWave) {
        const int j = LB.key[s];
        T.tj[s] = j;
        sd.cand[c0 + s] = j;
    }
    if (lane == 0) sd.cand_cnt[src] = total;
    __syncthreads();
    return total;
}

// Geodesics from the wavefront's sources to their candidate targets; writes
// their rows and returns whether any pair lies inside the guard band of the
// cutoff. Always inlined: the FP32-mixed kernel holds both precisions'
// loops, and a call to the FP64 one would make the FP32 loop spill registers
// around it.
template <typename R, class TL, int kG = 1>
__device__ __attribute__((always_inline)) inline unsigned run_sources(const GeoArgs &a, const SurfDesc &sd, TL &L,
                                                                  unsigned char *stk, int stk_bytes, const int *srcs,
                                                                  const int64_t *c0s, const int *ncs, int nsrc,
                                                                  bool guard_mode, int slot_id, SrcStats &st) {
    static_assert(kG == 1 || !TL::kBig, "groups: LDS tables only");
    constexpr int kB = kG == 1 ? TL::kBuckets : kGroupBuckets<kG>;  // hash buckets per source
    const int lane = lane_id();
    const long long t_start = clock64();
    const unsigned long long launches0 = st.launches;
    long long iters = 0, t_launch = 0;
    const bool fp32 = sizeof(R) == 4;
    // target ranges: a group's sources take 1/kG of the table each
    const int tspan = kG == 1 || nsrc == 1 ? 0 : kGroupCand<kG>;
    Ctx C;
    C.cutoff = sd.cutoff;
    // FP32 results may be off by rounding: everything within the guard band
    // above the cutoff is still propagated and recorded, so that pairs near
    // the cutoff are seen and recomputed in FP64
    C.lb_slack = fp32 ? fmax(a.gp.slack32, a.gp.guard_rel) * C.cutoff : 0.0;
    C.cut_acc = C.cutoff + C.lb_slack;
    C.tol = fp32 ? a.gp.cone_tol32 : a.gp.cone_tol;
    C.tie_rel = fp32 ? a.gp.tie_rel32 : a.gp.tie_rel;
    C.tie_dir = fp32 ? a.gp.tie_dir32 : a.gp.tie_dir;
    C.root_keep = fp32 ? 1.0 - a.gp.root_rel32 : 1.0;
    C.rc = {C.root_keep, C.tie_dir, C.tie_rel};
    C.nc = ncs[0];
    C.nc4 = (ncs[0] + 3) & ~3;
    // source q's target count padded to four (read from ncs where a lane's
    // source decides q: an array indexed per lane would live in scratch)
    auto nc4_of = [&](int q) { return kG == 1 ? C.nc4 : (ncs[q] + 3) & ~3; };
    const HeRec *__restrict__ he = sd.m.he;
    const BendTable G = bend_table(a.roots, a.rstride, slot_id, a.rcap);
    Stack<R> S;
    S.lds = reinterpret_cast<typename RecOf<R>::T *>(stk);
    S.kL = stk_bytes / (int)sizeof(typename RecOf<R>::T);
    S.glb = reinterpret_cast<typename RecOf<R>::T *>(reinterpret_cast<Rec64 *>(a.stack) +
                                                      (size_t)slot_id * a.gp.stack_cap);
    S.gcap = fp32 ? 2 * a.gp.stack_cap : a.gp.stack_cap;
    S.lsp = 0;
    S.gsp = 0;

    // ---- the seeding's source frames and edge records, loaded before the
    // table set-up so that their latency overlaps it. Lane 3 q + k takes edge
    // k of source q's face (the face frame: vertex 0 at the origin, vertex 1
    // on the x axis; vertex i at (px(i), py(i)); per-lane indices are
    // selects, not array indexing, which would put the frame in scratch
    // memory).
    struct SrcFrame {
        int src, fs;
        double b0, b1, b2, L, cx, cy, sx, sy;
        __device__ double px(int i) const { return i == 0 ? 0.0 : i == 1 ? L : cx; }
        __device__ double py(int i) const { return i == 2 ? cy : 0.0; }
        __device__ double sb(int i) const { return i == 0 ? b0 : i == 1 ? b1 : b2; }
    };
    auto frame_of = [&](int q) {
        SrcFrame F;
        F.src = kG == 1 ? srcs[0] : srcs[q];
        F.fs = sd.face[F.src];
        F.b0 = sd.bary[3 * (int64_t)F.src];
        F.b1 = sd.bary[3 * (int64_t)F.src + 1];
        F.b2 = sd.bary[3 * (int64_t)F.src + 2];
        const HeRec R0 = he[3 * F.fs];
        F.L = R0.L;
        F.cx = R0.cx;
        F.cy = R0.cy;
        F.sx = F.b1 * F.L + F.b2 * F.cx;
        F.sy = F.b2 * F.cy;
        return F;
    };
    const bool seed_act = lane < 3 * nsrc;
    const int seed_q = kG == 1 || !seed_act ? 0 : lane / 3, seed_k = seed_act ? lane - 3 * seed_q : 0;
    const SrcFrame seed_F = frame_of(seed_q);
    const HeRec seed_Rh = he[3 * seed_F.fs + seed_k];
    const int seed_pe = seed_act ? sd.m.pidx[sd.m.T[3 * seed_F.fs + seed_k]] : -1;

    // ---- LDS tables. The sources' targets are flattened over the lanes
    // (entry s of source q at table slot q tspan + s; e1..e3 end sources 0..2
    // in the flattened order), so that a group's loads go out together.
    for (int e = lane; e < TL::kBuckets; e += kWave) L.head[e] = -1;
    if (lane == 0) {
        L.B.npend = 0;
        L.B.ntouched = 0;
    }
    constexpr int kQ = kG == 1 ? 1 : kG;
    int en[kQ];  // source q's entries end at en[q] in the flattened order
    {
        int acc = 0;
#pragma unroll
        for (int t = 0; t < kQ; ++t) {
            if (t < nsrc) acc += ncs[t];
            en[t] = acc;
        }
    }
    const int ntot = en[kQ - 1];
    // source and slot of flattened entry k
    auto entry_of = [&](int k, int &q, int &s) {
        q = 0;
        s = k;
#pragma unroll
        for (int t = 0; t + 1 < kQ; ++t)
            if (k >= en[t]) {
                q = t + 1;
                s = k - en[t];
            }
    };
    __syncthreads();
    for (int k = lane; k < ntot; k += kWave) {
        int q, s0;
        entry_of(k, q, s0);
        const int s = q * tspan + s0;
        const int j = L.tj[s];
        const int f = sd.face[j];
        L.tface[s] = f;
        for (int d = 0; d < 3; ++d) {
            L.tb[s][d] = sd.bary[3 * (int64_t)j + d];
            L.cb[s][d] = sd.xyz[3 * (int64_t)j + d];
        }
        L.cb[s][3] = C.cut_acc;
        L.d1[s] = INFINITY;
        L.d2[s] = INFINITY;
        L.t1x[s] = 0.0;
        L.t1y[s] = 0.0;
        L.tnext[s] = atomicExch(&L.head[q * kB + hash_bits<kB>(f)], s);
    }
    if (lane < 4 * nsrc) {
        // padding of each source's bound table to a multiple of four: never reachable
        const int q = kG == 1 ? 0 : lane >> 2, r = lane & 3;
        const int nc = kG == 1 ? ncs[0] : ncs[q];
        if (nc + r < ((nc + 3) & ~3)) {
            const int s = q * tspan + nc + r;
            L.cb[s][0] = L.cb[s][1] = L.cb[s][2] = 0.0;
            L.cb[s][3] = -INFINITY;
        }
    }
    __syncthreads();

    bool overflow = false;
    int pruned = 0;

    // ---- seed from each source (root -1 - q, sg = 0), in FP64: lane 3 q + k
    // takes edge k of source q's face (its frame and records were loaded
    // above)
    {
        const bool act = seed_act;
        const int q = seed_q, k = seed_k;
        const SrcFrame &F = seed_F;
        const int hb = q * kB;
        if (act && k == 0) L.B.sface[q] = F.fs;
        // the targets in the source's own face (lane k = 0 of each source)
        {
            int slot = act && k == 0 ? first_in_face<TL, kB>(L, F.fs, hb) : -1;
            while (__ballot(slot >= 0)) {
                bool ok = slot >= 0;
                double d = 0, tx = 0, ty = 0;
                if (ok) {
                    double qx = L.tb[slot][1] * F.L + L.tb[slot][2] * F.cx;
                    double qy = L.tb[slot][2] * F.cy;
                    double dx = qx - F.sx, dy = qy - F.sy;
                    d = sqrt(dx * dx + dy * dy);
                    if (d > 0.0) {
                        tx = dx / d;
                        ty = dy / d;
                    }
                }
                target_update(L, C, ok, slot, d, tx, ty, INFINITY);
                if (ok) slot = next_in_face(L, slot, F.fs);
            }
        }
        Win<R> w, wa, wb;
        bool want = false, wantA = false, wantB = false;
        bool rok = false, on_edge = false;
        int rv = 0;
        double rd = 0, rtx = 0, rty = 0;
        if (act) {
            const HeRec &Rh = seed_Rh;
            const int k1 = k == 2 ? 0 : k + 1, k2 = k == 0 ? 2 : k - 1;  // (k + 1) % 3, (k + 2) % 3
            const double ex = (F.px(k1) - F.px(k)) / Rh.L, ey = (F.py(k1) - F.py(k)) / Rh.L;
            const int pe = seed_pe;
            if (pe >= 0) {
                double dx = F.px(k) - F.sx, dy = F.py(k) - F.sy;
                rd = sqrt(dx * dx + dy * dy);
                rok = rd < C.cut_acc;
                rv = bend_entry<kG>(pe, q);
                rtx = rd > 0 ? dx / rd : 0.0;
                rty = rd > 0 ? dy / rd : 0.0;
            }
            const double hx = F.sb(k1) * Rh.L + F.sb(k2) * Rh.cx, hy = F.sb(k2) * Rh.cy;
            if (Rh.twin >= 0) {
                w.px = (R)(Rh.L - hx);
                w.py = (R)(-hy);
                w.b0 = R(0);
                w.b1 = (R)Rh.L;
                w.sg = R(0);
                w.c = (R)(-ex);
                w.s = (R)(-ey);
                w.he = Rh.twin;
                w.root = -1 - q;
                if (F.sb(k2) > 0.0) {
                    want = seg_dist(Rh.L - hx, -hy, 0.0, Rh.L) < C.cut_acc;
                } else {
                    on_edge = true;
                    // source on this edge: the face across contains it as well
                    const He<R> Ht = load_he(sd.m, Rh.twin, R(0));
                    w.py = R(0);
                    double F3[3][3], U3[3][3];
                    face_xyz(sd.m, Rh.twin / 3, Rh.twin % 3, F3, U3);
                    children(Ht, w, 0.0, true, C, F3, U3, L, wa, wantA, wb, wantB, pruned, q * tspan, nc4_of(q));
                }
            }
        }
        bend_update(G, L.B, C.rc, rok, rv, rd, rtx, rty, INFINITY);
        // on-edge sources: targets and third vertex of the face across (rare:
        // one source at a time, when a lane has found one)
        for (int qs = 0; qs < nsrc && __ballot(on_edge) != 0; ++qs) {
            const SrcFrame E = frame_of(qs);
            const int hbs = qs * kB;
            for (int kk = 0; kk < 3; ++kk) {
                const int kk1 = kk == 2 ? 0 : kk + 1, kk2 = kk == 0 ? 2 : kk - 1;
                bool on = E.sb(kk2) <= 0.0 && he[3 * E.fs + kk].twin >= 0;
                if (!on) continue;  // wave-uniform
                const HeRec Rh = he[3 * E.fs + kk];
                const int t = Rh.twin, g = t / 3, m = t % 3;
                const HeRec Rt = he[t];
                const double ex = (E.px(kk1) - E.px(kk)) / Rh.L, ey = (E.py(kk1) - E.py(kk)) / Rh.L;
                const double c = -ex, sn = -ey;
                const double hx = E.sb(kk1) * Rh.L + E.sb(kk2) * Rh.cx;
                const double ptx = Rh.L - hx;
                int slot = lane < 1 ? first_in_face<TL, kB>(L, g, hbs) : -1;
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
                            tx = c * dx - sn * dy;
                            ty = sn * dx + c * dy;
                        }
                    }
                    target_update(L, C, ok, slot, d, tx, ty, INFINITY);
                    if (ok) slot = next_in_face(L, slot, g);
                }
                double dx = Rt.cx - ptx, dy = Rt.cy;
                double d = sqrt(dx * dx + dy * dy);
                const int pe =
                    lane == 0 && (Rt.opp_flags & 1) && d < C.cut_acc ? sd.m.pidx[Rt.opp_flags >> 1] : -1;
                bend_update(G, L.B, C.rc, pe >= 0, bend_entry<kG>(pe, qs), d, (c * dx - sn * dy) / d,
                            (sn * dx + c * dy) / d, INFINITY);
            }
        }
        S.push(want, w, overflow);
        S.push(wantA, wa, overflow);
        S.push(wantB, wb, overflow);
    }

    // ---- propagation
    const long long t_loop = clock64();
    const bool eager = a.gp.eager != 0;
    bool have = false;
    Win<R> w;
    unsigned long long nwin = 0;
    const unsigned long long max_win = (unsigned long long)a.gp.max_windows * (unsigned long long)nsrc;
    for (;;) {
        ++iters;
        if (__ballot(overflow)) overflow = true;
        if (overflow) break;
        st.depth = max(st.depth, S.lsp + S.gsp);
        bool busy = S.refill(have, w);
        // bend-vertex launches: eagerly whenever the table is dirty, else
        // once nothing is left to propagate
        if (L.B.npend > 0 && (eager || !busy)) {
            const long long t0 = clock64();
            launch_roots<R, TL, kG>(a, sd, L, G, C, S, st, tspan, ncs);
            t_launch += clock64() - t0;
            if (!busy) busy = S.refill(have, w);
        }
        if (!busy) {
            if (L.B.npend == 0) break;
            continue;
        }
        nwin += (unsigned long long)__popcll(__ballot(have));
        if (nwin > max_win) {
            overflow = true;
            break;
        }

        // ---- process the lane's window
        Win<R> cl, cr;
        bool hl = false, hr = false;
        He<R> H;
        double txc = 0.0;
        double F3[3][3], U3[3][3];
        double wtx = 0.0, wty = 0.0, wD2 = INFINITY;  // the root's tangent and other-direction distance
        int f = -1, k = 0;
        // the window's source: its targets, hash buckets and bend-vertex entries
        const int q = have ? slot_of<kG>(w.root) : 0;
        const int tb = q * tspan, hb = q * kB;
        if (have) {
            // the records depend only on the entry half-edge and the root:
            // issue them together
            f = w.he / 3;
            k = w.he % 3;
            H = load_he(sd.m, w.he, R(0));
            face_xyz(sd.m, f, k, F3, U3);
            double rD = 0.0, rL = INFINITY;
            if (w.root >= 0) {
                rD = G.rD[w.root];
                rL = G.rL[w.root];
                wtx = G.rtx[w.root];
                wty = G.rty[w.root];
                wD2 = G.rD2[w.root];
            }
            // stale: the window comes from an earlier launch of its root, or
            // the root has improved enough to be launched again (the same
            // test as the launch itself, so a root is never left without
            // live windows)
            if (w.root >= 0 && bend_stale(rD, rL, w, C.rc)) {
                have = false;
                ++st.stale;
            }
            txc = (double)w.px + ((double)H.cx - (double)w.px) * (-(double)w.py) / ((double)H.cy - (double)w.py);
        }
        // the third vertex's bend-vertex number, loaded now so that the target
        // queries cover its latency
        const int pv3 = have && H.pseudo ? sd.m.pidx[H.opp] : -1;
        // targets in face f
        {
            int slot = have ? first_in_face<TL, kB>(L, f, hb) : -1;
            while (__ballot(slot >= 0)) {
                bool ok = false;
                double d = 0, tx = 0, ty = 0, alt = INFINITY;
                if (slot >= 0) {
                    const R qx = (R)L.tb[slot][(k + 1) % 3] * H.L + (R)L.tb[slot][(k + 2) % 3] * H.cx;
                    const R qy = (R)L.tb[slot][(k + 2) % 3] * H.cy;
                    const R xq = w.px + (qx - w.px) * (-w.py) / (qy - w.py);
                    const R sl = (R)C.tol * H.L;
                    if (xq >= w.b0 - sl && xq <= w.b1 + sl) {
                        R dx = qx - w.px, dy = qy - w.py;
                        const R l = sqrt(dx * dx + dy * dy);
                        d = (double)w.sg + (double)l;
                        ok = d < C.cut_acc;
                        if (w.root < 0) {
                            dx /= l;
                            dy /= l;
                            tx = (double)(w.c * dx - w.s * dy);
                            ty = (double)(w.s * dx + w.c * dy);
                        } else {
                            tx = wtx;
                            ty = wty;
                            alt = wD2 + (double)l;
                        }
                    }
                }
                target_update(L, C, ok, slot, d, tx, ty, alt);
                if (slot >= 0) slot = next_in_face(L, slot, f);
            }
        }
        const int pe3 = pv3 >= 0 ? bend_entry<kG>(pv3, q) : -1;
        // third vertex as a bend vertex: the candidate now, its table entry
        // loaded now and applied after the children (whose arithmetic covers
        // the load's latency)
        bool ok3 = false;
        double d3 = 0, tx3 = 0, ty3 = 0, alt3 = INFINITY;
        BendEntry pE;
        {
            bool ok = false;
            double d = 0, tx = 0, ty = 0, alt = INFINITY;
            if (have && H.pseudo) {
                const double sl = C.tol * (double)H.L;
                if (txc >= (double)w.b0 - sl && txc <= (double)w.b1 + sl) {
                    R dx = H.cx - w.px, dy = H.cy - w.py;
                    const R l = sqrt(dx * dx + dy * dy);
                    d = (double)w.sg + (double)l;
                    ok = d < C.cut_acc;
                    if (w.root < 0) {
                        dx /= l;
                        dy /= l;
                        tx = (double)(w.c * dx - w.s * dy);
                        ty = (double)(w.s * dx + w.c * dy);
                    } else {
                        tx = wtx;
                        ty = wty;
                        alt = wD2 + (double)l;
                    }
                }
            }
            ok3 = ok;
            d3 = d;
            tx3 = tx;
            ty3 = ty;
            alt3 = alt;
            if (ok) pE = bend_load(G, pe3);
        }
        if (have) children(H, w, txc, false, C, F3, U3, L, cl, hl, cr, hr, pruned, tb, nc4_of(q));
        bend_update_loaded(G, L.B, C.rc, ok3, pe3, d3, tx3, ty3, alt3, pE);
        // keep one child in the lane, push the other
        S.push(hl && hr, cr, overflow);
        if (have) {
            if (hl) w = cl;
            else if (hr) w = cr;
            else have = false;
        }
    }

    // ---- results (rows of the candidate layout)
    const long long t_res = clock64();
    const bool ovf = __ballot(overflow) != 0;
    unsigned near_q = 0;  // bit q: a pair of source q lies inside the guard band
    // flattened over the sources' entries like the table (each lane takes
    // the 3D frame of its entry's source face)
    for (int k = lane; k < ntot; k += kWave) {
        int q, s;
        entry_of(k, q, s);
        const int tb = q * tspan;
        // the face frame: x along its first half-edge (the face record's unit
        // direction), y = normal x x
        const int fs = L.B.sface[q];
        const double *ux = sd.m.fpos + 18 * (int64_t)fs + 9;
        const double *nn = sd.m.fnrm + 3 * (int64_t)fs;
        const double ex3[3] = {ux[0], ux[1], ux[2]};
        const double ey3[3] = {nn[1] * ex3[2] - nn[2] * ex3[1], nn[2] * ex3[0] - nn[0] * ex3[2],
                               nn[0] * ex3[1] - nn[1] * ex3[0]};
        const int64_t o = (kG == 1 ? c0s[0] : c0s[q]) + s;
        double d = L.d1[tb + s];
        uint8_t fl = 0;
        if (ovf) d = NAN;
        if (L.d2[tb + s] - d <= C.tie_rel * d) fl |= GSIM_PAIR_TIE_BIT;
        if (d == 0.0) fl |= GSIM_PAIR_ZERO_BIT;
        if (guard_mode) fl |= GSIM_PAIR_GUARD_BIT;
        if (fabs(d - C.cutoff) <= a.gp.guard_rel * C.cutoff) near_q |= 1u << q;
        sd.cdist[o] = d;
        sd.cflags[o] = fl;
        for (int c = 0; c < 3; ++c) sd.ctan[3 * o + c] = L.t1x[tb + s] * ex3[c] + L.t1y[tb + s] * ey3[c];
    }
    for (int o = 32; o > 0; o >>= 1) near_q |= (unsigned)__shfl_xor((int)near_q, o);
    if (kG == 1 && sd.prof && lane == 0) {
        long long *qp = sd.prof + 8 * (int64_t)srcs[0];
        const long long t_end = clock64();
        qp[0] += t_end - t_start;
        qp[1] += iters;
        qp[2] += (long long)nwin;
        qp[3] += (long long)(st.launches - launches0);
        qp[4] += t_loop - t_start;
        qp[5] += t_res - t_loop - t_launch;
        qp[6] += t_launch;
        qp[7] += t_end - t_res;
    }
    st.windows += nwin;
    st.pruned += pruned;
    st.overflow |= ovf;
    bend_reset(G, L.B);
    return near_q;
}

// One source (the single-source instantiations).
template <typename R, class TL>
__device__ __attribute__((always_inline)) inline unsigned run_source(const GeoArgs &a, const SurfDesc &sd, TL &L,
                                                                 unsigned char *stk, int stk_bytes, int src, int64_t c0,
                                                                 int nc, bool guard_mode, int slot_id, SrcStats &st) {
    return run_sources<R, TL, 1>(a, sd, L, stk, stk_bytes, &src, &c0, &nc, 1, guard_mode, slot_id, st);
}

// The fused update of one source particle (lane 0): force from its row,
// integrator, walk, new state into the next-state arrays; returns its pair
// count (wc: the walk's counts). It runs after the source loop (a fused
// launch has one workgroup per source), where nothing of the propagation is
// live, so it costs the loop no registers.
__device__ __attribute__((always_inline)) inline int fused_move(const SurfDesc &sd, int src, WalkCounts &wc) {
    double F[3], E;
    int np = 0;
    row_force(src, sd.cand_cnt, sd.cap, sd.cdist, sd.ctan, sd.cutoff, sd.pkind, sd.pk, sd.psigma, F, E, np);
    move_particle(sd, src, F, sd.face_out, sd.bary_out, sd.vel_out, wc);
    return np;
}

// Two waves per SIMD: with up to eight workgroups' LDS on a compute unit, a
// wavefront may hold at most 256 registers.
// kMode 0: a persistent grid whose workgroups claim sources until none is
// left; 1: one workgroup per source (a launch with no more sources than
// resident slots), which carries no loop state through the propagation and
// compiles to fewer registers; 2: as 1, and the source particle is then moved
// (the fused update). Only mode 2 holds the update's code, which would
// otherwise change the register allocation of every launch.
// kBig: the big-candidate instantiation (targets in a per-wavefront global
// area, rows as wide as the surface's row capacity).
// kG = 2 or 4: the grouped instantiations (persistent grid, LDS tables): a
// wavefront claims kG sources at a time and propagates together those on
// the same surface with at most kGroupCand candidates each; a source with
// more runs alone over the whole table. In FP32-mixed mode the group runs in
// FP32 and each of its sources with a pair in the guard band again alone in
// FP64.
template <bool kMixed, int kStk, int kMode, bool kBig, int kG = 1>
__global__ __launch_bounds__(kWave, 2) void k_geodesic(GeoArgs a) {
    constexpr bool kOne = kMode >= 1, kFuse = kMode == 2;
    static_assert(kG == 1 || (kMode == 0 && !kBig), "groups: persistent LDS-table launches");
    __shared__ typename std::conditional<kBig, LdsBig, Lds>::type L;
    __shared__ alignas(16) unsigned char stk[kStk];
    const int lane = lane_id();
    const int total = a.bi.begin[a.bi.nsurf];
    int chunk = blockIdx.x % kChunks, chunks_left = kChunks;
    SrcStats st;
    st.windows = st.launches = st.stale = st.guards = 0;
    st.pruned = 0;
    st.depth = 0;
    st.overflow = false;
    unsigned long long c_limited = 0;
    unsigned long long fused_np = 0;  // neighbour pairs of the moved particle (lane 0)
    WalkCounts fused_wc = {0, 0, 0, 0, 0, 0};  // its walk's counts (lane 0)
    int fused_src = -1, fused_si = 0;  // the source a fused launch's workgroup took
    int next = 0, left = 0;  // claimed sources not yet processed
    if (kOne) {
        // one workgroup per source, no claims: workgroup b takes position
        // b / 8 of chunk b mod 8, where chunk c holds the sources of the
        // workgroups with b mod 8 = c (a bijection onto the sources in cell
        // order, each chunk a contiguous region)
        if ((int)blockIdx.x < total) {
            const int c = (int)blockIdx.x % kChunks;
            int start = 0;
            for (int k = 0; k < c; ++k) start += (total - k + kChunks - 1) / kChunks;
            next = start + (int)blockIdx.x / kChunks;
            left = 1;
        }
        chunks_left = 0;
    }
    for (;;) {
        // ---- next source: claim `grab` consecutive ones, XCD-local chunk first
        if (left == 0) {
            while (chunks_left > 0) {
                const int lo = (int)(((int64_t)total * chunk) / kChunks);
                const int hi = (int)(((int64_t)total * (chunk + 1)) / kChunks);
                int t = 0;
                if (lane == 0) t = atomicAdd(&a.work[chunk * kWorkStride], a.grab);
                t = __builtin_amdgcn_readlane(t, 0);
                if (lo + t < hi) {
                    next = lo + t;
                    left = min(a.grab, hi - next);
                    break;
                }
                chunk = (chunk + 1) % kChunks;
                --chunks_left;
            }
            if (left == 0) break;
        }
        const int idx = next++;
        --left;
        const int si = __builtin_amdgcn_readfirstlane(batch_surface(a.bi, idx));
        const SurfDesc &sd = a.sd[si];
        const int src = sd.order[idx - a.bi.begin[si]];
        if constexpr (kG > 1) {
            // up to kG sources of the claimed range on this surface, each
            // searched into its share of the table; those with no candidate
            // drop out, those with more than a share wait and run alone
            // over the whole table
            // the claimed sources that follow on the same surface
            const int more = min(kG - 1, min(left, a.bi.begin[si + 1] - next));
            next += more;
            left -= more;
            int nb, na;
            if (a.pre_cand) take_candidates<kG>(sd, L, idx - a.bi.begin[si], 1 + more, nb, na);
            else find_candidates_group<kG>(sd, L, idx - a.bi.begin[si], 1 + more, nb, na);
            // FP32-mixed: the group in FP32, then each source with a pair
            // inside the guard band of the cutoff again in FP64, alone
            if (nb > 0) {
                st.overflow = false;
                const unsigned nearm =
                    kMixed ? run_sources<float, Lds, kG>(a, sd, L, stk, kStk, L.gsrc, L.gc0, L.gnc, nb, false,
                                                         blockIdx.x, st)
                           : run_sources<double, Lds, kG>(a, sd, L, stk, kStk, L.gsrc, L.gc0, L.gnc, nb, false,
                                                          blockIdx.x, st);
                if (st.overflow) c_limited += (unsigned long long)nb;
                if constexpr (kMixed) {
                    for (int q = 0; q < nb; ++q) {
                        if (!((nearm >> q) & 1u)) continue;  // wave-uniform
                        const int s1 = L.gsrc[q];
                        const int64_t c = L.gc0[q];
                        const int n = a.pre_cand ? take_row(sd, L, s1, c) : find_candidates(sd, L, s1, c);
                        st.overflow = false;
                        run_sources<double, Lds, kG>(a, sd, L, stk, kStk, &s1, &c, &n, 1, true, blockIdx.x, st);
                        ++st.guards;
                        if (st.overflow) ++c_limited;
                    }
                }
            }
            for (int g = 0; g < na; ++g) {
                const int s1 = L.galone[g];
                const int64_t c = (int64_t)s1 * kMaxCand;
                const int n = a.pre_cand ? take_row(sd, L, s1, c) : find_candidates(sd, L, s1, c);
                if (n > kMaxCand) {
                    if (lane == 0) ++c_limited;
                } else {
                    st.overflow = false;
                    if (kMixed) {
                        if (run_sources<float, Lds, kG>(a, sd, L, stk, kStk, &s1, &c, &n, 1, false, blockIdx.x, st)) {
                            run_sources<double, Lds, kG>(a, sd, L, stk, kStk, &s1, &c, &n, 1, true, blockIdx.x, st);
                            ++st.guards;
                        }
                    } else {
                        run_sources<double, Lds, kG>(a, sd, L, stk, kStk, &s1, &c, &n, 1, false, blockIdx.x, st);
                    }
                    if (st.overflow) ++c_limited;
                }
            }
            continue;
        }
        // the propagation of one source over its target table
        auto process = [&](auto &T, int64_t c0, int nc, int cap) {
            if (nc > cap) {
                if (lane == 0) ++c_limited;
            } else if (nc > 0) {
                st.overflow = false;
                if (kMixed) {
                    // FP32 pass; a pair inside the guard band sends the source through FP64
                    if (run_source<float>(a, sd, T, stk, kStk, src, c0, nc, false, blockIdx.x, st)) {
                        run_source<double>(a, sd, T, stk, kStk, src, c0, nc, true, blockIdx.x, st);
                        ++st.guards;
                    }
                } else {
                    run_source<double>(a, sd, T, stk, kStk, src, c0, nc, false, blockIdx.x, st);
                }
                if (st.overflow) ++c_limited;
            }
        };
        if constexpr (kBig) {
            const int cap = min(sd.cap, min(a.gcap, kBigSort));
            const int64_t c0 = (int64_t)src * sd.cap;
            GTab T = gtab_of(a.gtab, a.gstride, blockIdx.x, a.gcap, L);
            const int nc = find_candidates_big(sd, L, T, src, c0, cap);
            process(T, c0, nc, cap);
        } else {
            const int64_t c0 = (int64_t)src * kMaxCand;
            const int nc = find_candidates(sd, L, src, c0);
            process(L, c0, nc, kMaxCand);
        }
        if (kOne) {
            // one source per workgroup (in mode 2 its particle is moved below)
            fused_src = src;
            fused_si = si;
            break;
        }
    }
    if (kFuse && fused_src >= 0) {
        // the row is final: move the source particle (the same force sum,
        // integrator and walk as the separate update kernel, read back from
        // the row this wavefront has just written) into the next-state
        // arrays, which no source reads during the pass
        __syncthreads();
        if (lane == 0) fused_np += (unsigned long long)fused_move(a.sd[fused_si], fused_src, fused_wc);
    }
    unsigned long long pr = (unsigned long long)st.pruned, sl = st.stale;
    for (int o = 32; o > 0; o >>= 1) {
        pr += __shfl_xor(pr, o);
        sl += __shfl_xor(sl, o);
    }
    Counters *ctr = a.ctr + ((int)blockIdx.x % kCtrSlots) * kCtrStride;
    if (lane == 0) {
        // only the counts that are not zero
        if (st.windows) atomicAdd(&ctr->windows, st.windows);
        if (pr) atomicAdd(&ctr->pruned, pr);
        if (st.launches) atomicAdd(&ctr->launches, st.launches);
        if (sl) atomicAdd(&ctr->stale, sl);
        if (c_limited) atomicAdd(&ctr->limited, c_limited);
        if (st.depth) atomicMax(&ctr->max_depth, (unsigned long long)st.depth);
        if (st.guards) atomicAdd(&ctr->guards, st.guards);
        if (fused_np) atomicAdd(&ctr->nbr_pairs, fused_np);
        if (fused_wc.nonfinite) atomicAdd(&ctr->nonfinite, 1ull);
        if (fused_wc.cross_n) atomicAdd(&ctr->crossings, (unsigned long long)fused_wc.cross_n);
    }
}

template <bool kMixed, int kStk, int kMode, bool kBig, int kG = 1>
void launch_one(int nslots, size_t pad, const GeoArgs &a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (ev0 || ev1)
        hipExtLaunchKernelGGL((k_geodesic<kMixed, kStk, kMode, kBig, kG>), dim3(nslots), dim3(kWave), (uint32_t)pad, s,
                              ev0, ev1, 0, a);
    else hipLaunchKernelGGL((k_geodesic<kMixed, kStk, kMode, kBig, kG>), dim3(nslots), dim3(kWave), pad, s, a);
}
// the grouped instantiations: persistent grid, LDS tables
template <bool kMixed, int kG>
void launch_groups(int kb, int nslots, size_t pad, const GeoArgs &a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (kb <= 4) launch_one<kMixed, 4096, 0, false, kG>(nslots, pad, a, s, ev0, ev1);
    else if (kb <= 8) launch_one<kMixed, 8192, 0, false, kG>(nslots, pad, a, s, ev0, ev1);
    else launch_one<kMixed, 16384, 0, false, kG>(nslots, pad, a, s, ev0, ev1);
}
template <bool kMixed, int kMode>
void launch_stack(int kb, bool big, int nslots, size_t pad, const GeoArgs &a, hipStream_t s, hipEvent_t ev0,
                  hipEvent_t ev1) {
    if (big) launch_one<kMixed, kBigStk, kMode, true>(nslots, pad, a, s, ev0, ev1);
    else if (kb <= 4) launch_one<kMixed, 4096, kMode, false>(nslots, pad, a, s, ev0, ev1);
    else if (kb <= 8) launch_one<kMixed, 8192, kMode, false>(nslots, pad, a, s, ev0, ev1);
    else launch_one<kMixed, 16384, kMode, false>(nslots, pad, a, s, ev0, ev1);
}
template <bool kMixed>
void launch_variant(int mode, int kb, bool big, int nslots, size_t pad, const GeoArgs &a, hipStream_t s,
                    hipEvent_t ev0, hipEvent_t ev1) {
    if (mode == 2) launch_stack<kMixed, 2>(kb, big, nslots, pad, a, s, ev0, ev1);
    else if (mode == 1) launch_stack<kMixed, 1>(kb, big, nslots, pad, a, s, ev0, ev1);
    else launch_stack<kMixed, 0>(kb, big, nslots, pad, a, s, ev0, ev1);
}

}  // namespace

hipError_t launch_geodesic(const SurfDesc *desc, const BatchIdx &bi, const GeoParams &gp, const GeoShape &shape,
                           char *stack_mem, char *roots, int64_t rstride, int rcap, int32_t *work_ctr, Counters *ctr,
                           bool fp32, bool fuse, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, char *gtab,
                           int gcap, int group, bool pre_cand) {
    GeoArgs a;
    a.sd = desc;
    a.bi = bi;
    a.gp = gp;
    a.stack = stack_mem;
    a.work = work_ctr;
    a.ctr = ctr;
    // one workgroup per source when there are no more sources than slots
    // (always so when fused: the update requires it)
    const int total = bi.begin[bi.nsurf];
    const int mode = fuse ? 2 : (total <= shape.nslots ? 1 : 0);
    a.grab = shape.grab < 1 || mode > 0 ? 1 : shape.grab;
    a.roots = roots;
    a.rstride = rstride;
    a.rcap = rcap;
    const bool big = gcap > 0;
    a.gtab = gtab;
    a.gstride = big ? gtab_bytes(gcap) : 0;
    a.gcap = gcap;
    a.pre_cand = pre_cand && group > 1 ? 1 : 0;

    if (shape.nslots < 1 || total < 1) return hipSuccess;
    if (fuse && total > shape.nslots) return hipErrorInvalidValue;  // the fused update needs a slot per source
    if (big && (!gtab || gcap > kBigCandMax)) return hipErrorInvalidValue;
    const size_t pad = shape.pad_lds > 0 ? (size_t)shape.pad_lds : 0;
    if (group > 1) {
        // several sources per wavefront: persistent grid, LDS tables, claims
        // of a multiple of the group so that groups come from one claimed
        // range
        if ((group != 2 && group != 4 && group != 8) || big || mode != 0 || rcap % group) return hipErrorInvalidValue;
        a.grab = group * a.grab;
        if (fp32) {
            if (group == 2) launch_groups<true, 2>(shape.lds_stack_kb, shape.nslots, pad, a, s, ev0, ev1);
            else if (group == 4) launch_groups<true, 4>(shape.lds_stack_kb, shape.nslots, pad, a, s, ev0, ev1);
            else launch_groups<true, 8>(shape.lds_stack_kb, shape.nslots, pad, a, s, ev0, ev1);
        } else {
            if (group == 2) launch_groups<false, 2>(shape.lds_stack_kb, shape.nslots, pad, a, s, ev0, ev1);
            else if (group == 4) launch_groups<false, 4>(shape.lds_stack_kb, shape.nslots, pad, a, s, ev0, ev1);
            else launch_groups<false, 8>(shape.lds_stack_kb, shape.nslots, pad, a, s, ev0, ev1);
        }
        return hipGetLastError();
    }
    if (fp32) launch_variant<true>(mode, shape.lds_stack_kb, big, shape.nslots, pad, a, s, ev0, ev1);
    else launch_variant<false>(mode, shape.lds_stack_kb, big, shape.nslots, pad, a, s, ev0, ev1);
    return hipGetLastError();
}

hipError_t launch_candidates(const SurfDesc *desc, const BatchIdx &bi, int group, hipStream_t s) {
    const int total = bi.begin[bi.nsurf];
    if (total <= 0) return hipSuccess;
    const int nb = (total + group - 1) / group;
    if (group == 2) hipLaunchKernelGGL(k_candidates<2>, dim3(nb), dim3(kWave), 0, s, desc, bi);
    else if (group == 4) hipLaunchKernelGGL(k_candidates<4>, dim3(nb), dim3(kWave), 0, s, desc, bi);
    else if (group == 8) hipLaunchKernelGGL(k_candidates<8>, dim3(nb), dim3(kWave), 0, s, desc, bi);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

int geodesic_blocks_per_cu(int lds_stack_kb, bool fp32, bool big) {
    int nb = 0;
    const void *f;
    if (big) f = fp32 ? (const void *)&k_geodesic<true, kBigStk, 0, true> : (const void *)&k_geodesic<false, kBigStk, 0, true>;
    else if (lds_stack_kb <= 4)
        f = fp32 ? (const void *)&k_geodesic<true, 4096, 0, false> : (const void *)&k_geodesic<false, 4096, 0, false>;
    else if (lds_stack_kb <= 8)
        f = fp32 ? (const void *)&k_geodesic<true, 8192, 0, false> : (const void *)&k_geodesic<false, 8192, 0, false>;
    else f = fp32 ? (const void *)&k_geodesic<true, 16384, 0, false> : (const void *)&k_geodesic<false, 16384, 0, false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kWave, 0) != hipSuccess) return 0;
    return nb;
}

size_t geodesic_lds_bytes(int lds_stack_kb, bool, bool big) {
    if (big) return sizeof(LdsBig) + (size_t)kBigStk;
    const int kb = lds_stack_kb <= 4 ? 4 : (lds_stack_kb <= 8 ? 8 : 16);
    return sizeof(Lds) + (size_t)kb * 1024;
}

int64_t geodesic_gtab_bytes(int gcap) { return gtab_bytes(gcap); }


}  // namespace gsim
