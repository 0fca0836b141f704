// All-pairs exact polyhedral geodesics (no cutoff), one source per wave64.
//
// Every other particle of the surface is a target, so a source's windows
// must cover the whole mesh (the paper's full-mesh sequence trees, Sec. 3.1
// and Sec. 4; the Thomson-like long-range case). Without a cutoff two things
// keep the unfolding finite, both exact:
//  - vertex domination (the window filter of Xin and Wang's improvement of
//    the Chen-Han algorithm, the method the paper uses): each source keeps a
//    table D(v) of path lengths that have reached every vertex. A child window
//    on an edge S-E whose distance function f(x) = sg + |p - x| exceeds
//    D(S) + x (the path through S, then along the edge) is dominated there;
//    since f(x) - x is non-increasing the dominated part is [x0, x*) and is
//    trimmed (likewise (x**, x1] for the path through E). A window dominated
//    everywhere is dropped. Shortest paths to points beyond the edge are
//    never dominated this way, so no pair is lost.
//  - processing in rounds of increasing key: children whose key reaches the
//    round's threshold wait for the next round, so the search cannot run
//    ahead along one branch; once every target has been reached, windows
//    whose key exceeds the largest target distance (widened by the tie gap)
//    are dropped.
// Bend vertices are launched by the rules of the cutoff kernel, from a table
// that can hold every saddle and boundary vertex of the surface.
//
// Mapping: the state of all n targets (best distance, best distance of
// another direction, tangent; 32 bytes each), the vertex table, the
// bend-vertex table and the window overflow in per-wavefront global areas
// (the overflow is two-ended: the current round grows from one end, the next
// round from the other); targets are found through the surface's
// particles-by-face index.
#include <cmath>

#include "gsim_internal.h"
#include "window.h"

namespace gsim {
namespace {

using namespace wnd;

constexpr int kChunks = 8;
static_assert(kChunks == kWorkChunks, "one work counter per chunk");

struct AllArgs {
    const SurfDesc *sd;
    BatchIdx bi;
    GeoParams gp;
    void *stack;     // per wavefront: stack_cap records of 64 bytes
    double *vdist;   // per wavefront: vstride vertex distances
    int64_t vstride;
    char *roots;     // per wavefront: a bend-vertex table (rstride bytes, rcap vertices)
    int64_t rstride;
    int rcap;
    int32_t *work;
    Counters *ctr;
    double2 *ttab;   // per wavefront: tcap target distances (best, tie), then tcap tangents
    int tcap;
    int grab;
};

struct AllLds {
    BendLds B;
    int32_t unfound;  // targets not reached yet
    double maxb;      // windows with a larger key cannot improve any target
};

// Per-source constants.
struct ACtx {
    double tol, tie_rel, tie_dir, root_keep, dom_rel, bucket;
    double cutoff;  // infinity for all pairs
    RootCfg rc;
};

struct SrcStats {
    unsigned long long windows, launches, stale, guards;
    int pruned, depth;
    bool overflow;
};

// Window stack of the round-by-round order: LDS first, then one end of the
// wavefront's global area for the current round; the next round's windows
// grow from the other end.
template <typename R>
struct RoundStack {
    using Rec = typename RecOf<R>::T;
    int kL;
    Rec *lds;
    Rec *glb;
    int gcap;
    int lsp, gsp, dsp;
    int dir;

    __device__ Rec &cur(int k) { return dir == 0 ? glb[k] : glb[gcap - 1 - k]; }
    __device__ Rec &def(int k) { return dir == 0 ? glb[gcap - 1 - k] : glb[k]; }

    __device__ void push(bool want, bool later, const Win<R> &w, bool &overflow) {
        const bool now = want && !later;
        uint64_t m = __ballot(now);
        int cnt = __popcll(m);
        if (cnt) {
            const int r = __popcll(m & lanemask_lt());
            const int space = kL - lsp;
            if (now) {
                if (r < space) {
                    store_rec(lds[lsp + r], w);
                } else {
                    const int pos = gsp + (r - space);
                    if (pos + dsp < gcap) store_rec(cur(pos), w);
                    else overflow = true;
                }
            }
            const int to_l = min(cnt, space);
            lsp += to_l;
            gsp = min(gsp + (cnt - to_l), gcap - dsp);
        }
        const bool lat = want && later;
        m = __ballot(lat);
        cnt = __popcll(m);
        if (cnt) {
            const int r = __popcll(m & lanemask_lt());
            if (lat) {
                const int pos = dsp + r;
                if (pos + gsp < gcap) store_rec(def(pos), w);
                else overflow = true;
            }
            dsp = min(dsp + cnt, gcap - gsp);
        }
    }
    __device__ bool refill(bool &have, Win<R> &w) {
        const uint64_t need = __ballot(!have);
        const int nneed = __popcll(need);
        const int r = __popcll(need & lanemask_lt());
        const int take_l = min(nneed, lsp);
        if (!have && r < take_l) {
            load_rec(lds[lsp - 1 - r], w);
            have = true;
        }
        lsp -= take_l;
        if (nneed > take_l && gsp > 0) {
            __syncthreads();  // make earlier global pushes of other lanes visible
            const int take_g = min(nneed - take_l, gsp);
            if (!have && r >= take_l && r < take_l + take_g) {
                load_rec(cur(gsp - 1 - (r - take_l)), w);
                have = true;
            }
            gsp -= take_g;
        }
        return __ballot(have) != 0;
    }
    // the next round's windows become the current ones (the current round is empty)
    __device__ void next_round() {
        dir ^= 1;
        gsp = dsp;
        dsp = 0;
    }
};

// Path length reaching a vertex: the table keeps the minimum (positive
// doubles order like their bit patterns).
__device__ inline void vdist_min(double *Dv, int v, double d) {
    atomicMin(reinterpret_cast<unsigned long long *>(Dv + v), (unsigned long long)__double_as_longlong(d));
}

// Target update: best distance, its tangent, and the best distance among
// candidates whose direction differs (tie gap); `alt` is the distance of an
// another-direction path that comes with the candidate. The lanes load their
// targets together and leave when their candidate cannot change anything
// (the stored distances only decrease); the others are applied one lane at a
// time in registers, each result passed to every lane holding the same
// target, and written back once (the tangent only where the best distance
// fell).
__device__ inline void target_update(AllLds &L, double2 *td, double2 *tt, const ACtx &C, bool ok, int j, double d,
                                     double tx, double ty, double alt) {
    double c1 = INFINITY, c2 = INFINITY;
    if (ok) {
        const double2 c = td[j];
        c1 = c.x;
        c2 = c.y;
        if (d >= c1 && d >= c2 && alt >= c2) ok = false;
    }
    uint64_t m = __ballot(ok);
    if (!m) return;
    const double c1_in = c1, c2_in = c2;
    double ax = 0.0, ay = 0.0;
    if (ok && c1 < INFINITY) {
        const double2 t = tt[j];
        ax = t.x;
        ay = t.y;
    }
    int reached = 0;  // targets found for the first time
    // lanes on different targets (the usual case) update at once, else one
    // lane at a time
    bool dup = false;
    for (uint64_t r = m; r; r &= r - 1) {
        const int l = __ffsll((unsigned long long)r) - 1;
        dup |= ok && j == __builtin_amdgcn_readlane(j, l) && lane_id() != l;
    }
    if (!__ballot(dup)) {
        int first = 0;
        if (ok) {
            const bool found = c1 < INFINITY;
            const bool differ = !found || fabs(ax * ty - ay * tx) > C.tie_dir || ax * tx + ay * ty < 0.0;
            if (d < c1) {
                if (differ) c2 = fmin(c2, c1);
                c1 = d;
                ax = tx;
                ay = ty;
                first = !found;
            } else if (differ) {
                c2 = fmin(c2, d);
            }
            c2 = fmin(c2, alt);
        }
        reached = __popcll(__ballot(first));
        m = 0;
    }
    while (m) {
        const int l = __ffsll((unsigned long long)m) - 1;
        int first = 0;
        if (lane_id() == l) {
            const bool found = c1 < INFINITY;
            const bool differ = !found || fabs(ax * ty - ay * tx) > C.tie_dir || ax * tx + ay * ty < 0.0;
            if (d < c1) {
                if (differ) c2 = fmin(c2, c1);
                c1 = d;
                ax = tx;
                ay = ty;
                first = !found;
            } else if (differ) {
                c2 = fmin(c2, d);
            }
            c2 = fmin(c2, alt);
        }
        reached += __builtin_amdgcn_readlane(first, l);
        const int jl = __builtin_amdgcn_readlane(j, l);
        const double b1 = readlane_d(c1, l), b2 = readlane_d(c2, l);
        const double bx = readlane_d(ax, l), by = readlane_d(ay, l);
        if (ok && j == jl) {
            c1 = b1;
            c2 = b2;
            ax = bx;
            ay = by;
        }
        m &= m - 1;
    }
    if (ok) {
        if (c1 < c1_in || c2 < c2_in) td[j] = make_double2(c1, c2);
        if (c1 < c1_in) tt[j] = make_double2(ax, ay);
    }
    if (lane_id() == 0 && reached) L.unfound -= reached;
    lane_step_barrier();
}

// Trim a child interval [x0, x1] on an edge S -> E (length Lc, child frame
// origin S) against the paths through S and through E; returns false when
// nothing is left. f(x) = sg + |p - (x, 0)|. The path through S and then
// along the edge has length DS + x; it is shorter than the window where
// g(x) = f(x) - x - DS > 0, and g is non-increasing, so the dominated part
// is [x0, x*). Likewise h(x) = f(x) - (Lc - x) - DE is non-decreasing and
// the part dominated by the path through E is (x**, x1]. The vertex path
// lengths are widened by the factor 1 + rel first, so only parts dominated
// beyond the rounding error of the working precision are cut. f0 and f1
// return f at the final ends (each square root is taken once per end).
__device__ inline bool vertex_trim(double px, double py, double sg, double Lc, double DS, double DE, double rel,
                                   double &x0, double &x1, double &f0, double &f1) {
    // the vertex paths count as shorter only by more than `rel` of their length
    DS *= 1.0 + rel;
    DE *= 1.0 + rel;
    const double eps_x = 1e-9 * Lc;
    auto f = [&](double x) { return sg + sqrt((x - px) * (x - px) + py * py); };
    f0 = f(x0);
    f1 = f(x1);
    if (DS < INFINITY) {
        if (f1 - x1 - DS > 0.0) return false;
        if (f0 - x0 - DS > 0.0) {
            // g(x*) = 0: sqrt((x - px)^2 + py^2) = dl + x, dl = DS - sg
            const double dl = DS - sg;
            const double den = 2.0 * (px + dl);
            if (den > 0.0) {
                const double xs = (px * px + py * py - dl * dl) / den;
                if (xs - eps_x > x0) {
                    x0 = fmin(x1, xs - eps_x);
                    f0 = f(x0);
                }
            }
        }
    }
    if (DE < INFINITY) {
        if (f0 - (Lc - x0) - DE > 0.0) return false;
        if (f1 - (Lc - x1) - DE > 0.0) {
            // h(x**) = 0: sqrt((x - px)^2 + py^2) = mm - x, mm = DE + Lc - sg
            const double mm = DE + Lc - sg;
            const double den = 2.0 * (px - mm);
            if (den < 0.0) {
                const double xs = (px * px + py * py - mm * mm) / den;
                if (xs + eps_x < x1) {
                    x1 = fmax(x0, xs + eps_x);
                    f1 = f(x1);
                }
            }
        }
    }
    return x1 - x0 > 1e-12 * Lc;
}

// Is the whole child interval [x0, x1] dominated by the path through the
// face's third vertex O (at (ox, oy) in the child frame, on the near side of
// the edge), i.e. DO + |O - X| < f(X)? The points of the edge line where that
// holds are the line's intersection with one branch region of a hyperbola
// with foci p and O, which is convex: domination at both ends means
// domination everywhere in between. f0, f1: f at the two ends. The test at
// a point compares squares (f - DO > 0 and |O - X|^2 < (f - DO)^2): no
// square root, and its rounding stays far inside the widening by rel.
__device__ inline bool opposite_dominates(double ox, double oy, double DO, double rel, double x0, double x1, double f0,
                                          double f1) {
    if (!(DO < INFINITY)) return false;
    DO *= 1.0 + rel;
    auto dom = [&](double x, double f) {
        const double r = f - DO;
        return r > 0.0 && (x - ox) * (x - ox) + oy * oy < r * r;
    };
    return dom(x0, f0) && dom(x1, f1);
}

// Key (smallest distance) of a child window on [x0, x1] whose distance at
// the ends is f0, f1. In FP64 the ends are the window's own, so the key
// reuses them; FP32 windows take it from their rounded fields.
template <typename R>
__device__ inline double child_key(const Win<R> &c, double f0, double f1) {
    if constexpr (sizeof(R) == 8) {
        return c.px < c.b0 ? f0 : (c.px > c.b1 ? f1 : c.sg + fabs(c.py));
    } else {
        return (double)c.sg + (double)seg_dist(c.px, c.py, c.b0, c.b1);
    }
}

// Targets in face g (entry half-edge slot k of g) seen through window w.
template <typename R>
__device__ inline void query_face(const SurfDesc &sd, AllLds &L, const BendTable &G, double2 *td, double2 *tt,
                                  const ACtx &C, bool have, int src, int g, int k, const He<R> &H,
                                  const Win<R> &w) {
    int q = 0, q1 = 0;
    if (have) {
        q = sd.fstart[g];
        q1 = sd.fstart[g + 1];
    }
    while (__ballot(q < q1)) {
        bool ok = false;
        int j = 0;
        double d = 0, tx = 0, ty = 0, alt = INFINITY;
        if (q < q1) {
            j = sd.forder[q];
            if (j != src) {
                const double *b = sd.bary + 3 * (int64_t)j;
                const R qx = (R)b[(k + 1) % 3] * H.L + (R)b[(k + 2) % 3] * H.cx;
                const R qy = (R)b[(k + 2) % 3] * H.cy;
                const R xq = w.px + (qx - w.px) * (-w.py) / (qy - w.py);
                const R sl = (R)C.tol * H.L;
                if (xq >= w.b0 - sl && xq <= w.b1 + sl) {
                    R dx = qx - w.px, dy = qy - w.py;
                    const R l = sqrt(dx * dx + dy * dy);
                    d = (double)w.sg + (double)l;
                    ok = true;
                    if (w.root < 0) {
                        dx /= l;
                        dy /= l;
                        tx = (double)(w.c * dx - w.s * dy);
                        ty = (double)(w.s * dx + w.c * dy);
                    } else {
                        tx = G.rtx[w.root];
                        ty = G.rty[w.root];
                        alt = G.rD2[w.root] + (double)l;
                    }
                }
            }
            ++q;
        }
        target_update(L, td, tt, C, ok, j, d, tx, ty, alt);
    }
}

// Launch the pending bend vertices (their distance improved, or their best
// direction changed, or a tie appeared), their fans flattened over the lanes
// a chunk of vertices at a time.
template <typename R>
__device__ void launch_roots(const AllArgs &a, const SurfDesc &sd, AllLds &L, const BendTable &G, double2 *td,
                             double2 *tt, double *Dv, const ACtx &C, RoundStack<R> &S,
                             double T, int src, SrcStats &st) {
    const int lane = lane_id();
    const DevMesh &M = sd.m;
    const HeRec *__restrict__ he = M.he;
    // take the pending list (its vertices may be queued again while they launch)
    const int npend = L.B.npend;
    int nsel = 0;
    for (int base = 0; base < npend; base += kWave) {
        const int k = base + lane;
        int e = 0;
        bool sel = false;
        double D = 0.0;
        if (k < npend) {
            e = G.pend[k];
            D = G.rD[e];
            sel = D < G.rL[e] * C.rc.keep && D < L.maxb;
            G.queued[e] = 0;
        }
        const uint64_t mk = __ballot(sel);
        if (sel) {
            G.sel[nsel + __popcll(mk & lanemask_lt())] = e;
            G.rL[e] = D;
        }
        nsel += __popcll(mk);
    }
    if (lane == 0) L.B.npend = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nsel; c0 += kLaunchChunk) {
        const int cn = min(kLaunchChunk, nsel - c0);
        int carry = 0;
        for (int base = 0; base < cn; base += kWave) {
            const int k = base + lane;
            int deg = 0;
            if (k < cn) {
                const int e = G.sel[c0 + k];
                const int v = M.pvert[e];
                L.B.sel[k] = e;
                deg = M.fan_off[v + 1] - M.fan_off[v];
            }
            int inc = deg;
            for (int o = 1; o < kWave; o <<= 1) {
                const int y = __shfl_up(inc, o);
                if (lane >= o) inc += y;
            }
            if (k < cn) L.B.pref[k + 1] = carry + inc;
            st.launches += (unsigned long long)__popcll(__ballot(deg > 0));
            carry += __shfl(inc, kWave - 1);
        }
        if (lane == 0) L.B.pref[0] = 0;
        __syncthreads();
        const int total = carry;
        for (int base = 0; base < total; base += kWave) {
            const int idx = base + lane;
            const bool act = idx < total;
            int k = 0;
            if (act) {
                int lo = 0, hi = cn - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (L.B.pref[mid] <= idx) lo = mid;
                    else hi = mid - 1;
                }
                k = lo;
            }
            const int el = act ? L.B.sel[k] : 0;
            const int v = act ? M.pvert[el] : 0;
            const double D = act ? G.rD[el] : 0.0;
            const double vtx = act ? G.rtx[el] : 0.0, vty = act ? G.rty[el] : 0.0;
            const double D2 = act ? G.rD2[el] : INFINITY;
            const int h = act ? M.fan[M.fan_off[v] + (idx - L.B.pref[k])] : 0;
            const int hn = h - h % 3 + (h % 3 + 1) % 3;
            const HeRec Rh = he[h], Rn = he[hn];
            Win<R> nw;
            bool want = false;
            double key = 0.0;
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
                key = D + seg_dist(px, py, 0.0, Rn.L);
                want = key < L.maxb;
            }
            // direct targets in face(h): straight segments inside the face
            const int g = h / 3;
            int q = 0, q1 = 0;
            if (act) {
                q = sd.fstart[g];
                q1 = sd.fstart[g + 1];
            }
            const double *pv = M.V + 3 * (int64_t)v;
            while (__ballot(q < q1)) {
                bool ok = false;
                int j = 0;
                double d = 0;
                if (q < q1) {
                    j = sd.forder[q];
                    if (j != src) {
                        const double *b = sd.bary + 3 * (int64_t)j;
                        const int32_t *Tg = M.T + 3 * (int64_t)g;
                        double x[3] = {0, 0, 0};
                        for (int c = 0; c < 3; ++c)
                            for (int dd = 0; dd < 3; ++dd) x[dd] += b[c] * M.V[3 * (int64_t)Tg[c] + dd];
                        const double dx = x[0] - pv[0], dy = x[1] - pv[1], dz = x[2] - pv[2];
                        d = D + sqrt(dx * dx + dy * dy + dz * dz);
                        ok = true;
                    }
                    ++q;
                }
                target_update(L, td, tt, C, ok, j, d, vtx, vty, D2 + (d - D));
            }
            // the two other vertices of face(h), reached along its edges
            const int u1 = Rh.head, u2 = Rh.opp_flags >> 1;
            if (act) {
                vdist_min(Dv, u1, D + Rh.L);
                vdist_min(Dv, u2, D + Rh.Lp);
            }
            const int e1 = act ? M.pidx[u1] : -1;
            bend_update(G, L.B, C.rc, e1 >= 0, e1, D + Rh.L, vtx, vty, D2 + Rh.L);
            const int e2 = act ? M.pidx[u2] : -1;
            bend_update(G, L.B, C.rc, e2 >= 0, e2, D + Rh.Lp, vtx, vty, D2 + Rh.Lp);
            S.push(want, key >= T, nw, st.overflow);
        }
        __syncthreads();  // the chunk arrays are rewritten by the next chunk
    }
}

// One source's whole-mesh propagation and its row of results. With a
// finite cutoff, windows whose key reaches it are dropped (in FP32 a little
// beyond it, by the acceptance slack) and the row keeps every target; the
// pairs at or beyond the cutoff are left out downstream. Returns whether an
// FP32 result lies within the guard band around the cutoff (the caller then
// recomputes the source in FP64; `guard` marks that recompute). Inlined:
// as a call, the FP32 kernel spills around it and holds one wave per SIMD.
template <typename R>
__device__ __attribute__((always_inline)) inline bool run_all(const AllArgs &a, const SurfDesc &sd, AllLds &L,
                                                              double2 *td, double2 *tt, unsigned char *stk,
                                                              int stk_bytes, int src, int slot, bool guard,
                                                              SrcStats &st) {
    const int lane = lane_id();
    const bool fp32 = sizeof(R) == 4;
    const int n = sd.n;
    const DevMesh &M = sd.m;
    const HeRec *__restrict__ he = M.he;
    ACtx C;
    C.tol = fp32 ? a.gp.cone_tol32 : a.gp.cone_tol;
    C.tie_rel = fp32 ? a.gp.tie_rel32 : a.gp.tie_rel;
    C.tie_dir = fp32 ? a.gp.tie_dir32 : a.gp.tie_dir;
    C.root_keep = fp32 ? 1.0 - a.gp.root_rel32 : 1.0;
    C.rc = {C.root_keep, C.tie_dir, C.tie_rel};
    C.dom_rel = fp32 ? a.gp.dom_rel32 : a.gp.dom_rel;
    // rounds: wide ones mean fewer round changes, but on a surface with bend
    // vertices they launch vertices before their distances settle
    C.bucket = a.gp.bucket > 0.0 ? a.gp.bucket : (M.n_pseudo > 0 ? 4.0 : 16.0) * M.max_edge;
    C.cutoff = sd.cutoff;
    double *Dv = a.vdist + (int64_t)slot * a.vstride;
    const BendTable G = bend_table(a.roots, a.rstride, slot, a.rcap);
    RoundStack<R> S;
    S.lds = reinterpret_cast<typename RecOf<R>::T *>(stk);
    S.kL = stk_bytes / (int)sizeof(typename RecOf<R>::T);
    S.glb = reinterpret_cast<typename RecOf<R>::T *>(reinterpret_cast<Rec64 *>(a.stack) + (size_t)slot * a.gp.stack_cap);
    S.gcap = fp32 ? 2 * a.gp.stack_cap : a.gp.stack_cap;
    S.lsp = S.gsp = S.dsp = 0;
    S.dir = 0;

    // ---- tables
    for (int v = lane; v < M.nv; v += kWave) Dv[v] = INFINITY;
    for (int j = lane; j < n; j += kWave) {
        td[j] = make_double2(INFINITY, INFINITY);
        tt[j] = make_double2(0.0, 0.0);
    }
    if (lane == 0) {
        L.B.npend = 0;
        L.B.ntouched = 0;
        L.unfound = n - 1;
        L.maxb = C.cutoff < INFINITY ? C.cutoff * (fp32 ? 1.0 + fmax(a.gp.slack32, a.gp.guard_rel) : 1.0)
                                     : INFINITY;
    }
    __threadfence_block();
    __syncthreads();
    bool overflow = false;
    double T = C.bucket;

    // ---- seed from the source (root -1, sg = 0), in FP64
    const int fs = sd.face[src];
    const double sb[3] = {sd.bary[3 * (int64_t)src], sd.bary[3 * (int64_t)src + 1], sd.bary[3 * (int64_t)src + 2]};
    const HeRec R0 = he[3 * fs];
    const double P[3][2] = {{0.0, 0.0}, {R0.L, 0.0}, {R0.cx, R0.cy}};
    const double sx = sb[1] * P[1][0] + sb[2] * P[2][0], sy = sb[1] * P[1][1] + sb[2] * P[2][1];
    {
        // targets in the source's face: straight segments
        int q = lane == 0 ? sd.fstart[fs] : 0, q1 = lane == 0 ? sd.fstart[fs + 1] : 0;
        while (__ballot(q < q1)) {
            bool ok = false;
            int j = 0;
            double d = 0, tx = 0, ty = 0;
            if (q < q1) {
                j = sd.forder[q];
                if (j != src) {
                    const double *b = sd.bary + 3 * (int64_t)j;
                    const double qx = b[1] * P[1][0] + b[2] * P[2][0], qy = b[1] * P[1][1] + b[2] * P[2][1];
                    const double dx = qx - sx, dy = qy - sy;
                    d = sqrt(dx * dx + dy * dy);
                    if (d > 0.0) {
                        tx = dx / d;
                        ty = dy / d;
                    }
                    ok = true;
                }
                ++q;
            }
            target_update(L, td, tt, C, ok, j, d, tx, ty, INFINITY);
        }
    }
    {
        Win<R> w, wa, wb;
        bool want = false, wantA = false, wantB = false;
        int rv = -1;
        double rd = 0, rtx = 0, rty = 0;
        double ka = 0, kb = 0;
        if (lane < 3) {
            const int k = lane, h = 3 * fs + k;
            const HeRec Rh = he[h];
            const double ex = (P[(k + 1) % 3][0] - P[k][0]) / Rh.L, ey = (P[(k + 1) % 3][1] - P[k][1]) / Rh.L;
            const int v = M.T[h];
            {
                const double dx = P[k][0] - sx, dy = P[k][1] - sy;
                rd = sqrt(dx * dx + dy * dy);
                vdist_min(Dv, v, rd);
                rv = M.pidx[v];
                if (rv >= 0) {
                    rtx = rd > 0 ? dx / rd : 0.0;
                    rty = rd > 0 ? dy / rd : 0.0;
                }
            }
            const double hx = sb[(k + 1) % 3] * Rh.L + sb[(k + 2) % 3] * Rh.cx, hy = sb[(k + 2) % 3] * Rh.cy;
            if (Rh.twin >= 0) {
                w.px = (R)(Rh.L - hx);
                w.py = (R)(-hy);
                w.b0 = R(0);
                w.b1 = (R)Rh.L;
                w.sg = R(0);
                w.c = (R)(-ex);
                w.s = (R)(-ey);
                w.he = Rh.twin;
                w.root = -1;
                if (sb[(k + 2) % 3] > 0.0) {
                    want = true;
                } else {
                    // source on this edge: the face across contains it as well
                    const He<R> Ht = load_he(M, Rh.twin, R(0));
                    w.py = R(0);
                    if (Ht.tp >= 0) {
                        make_left(Ht, w, 0.0, (double)Ht.Lp, wa);
                        wantA = true;
                        ka = (double)seg_dist(wa.px, wa.py, wa.b0, wa.b1);
                    }
                    if (Ht.tn >= 0) {
                        make_right(Ht, w, 0.0, (double)Ht.Ln, wb);
                        wantB = true;
                        kb = (double)seg_dist(wb.px, wb.py, wb.b0, wb.b1);
                    }
                }
            }
        }
        bend_update(G, L.B, C.rc, rv >= 0, rv, rd, rtx, rty, INFINITY);
        // on-edge sources: targets and third vertex of the face across
        for (int k = 0; k < 3; ++k) {
            const bool on = sb[(k + 2) % 3] <= 0.0 && he[3 * fs + k].twin >= 0;
            if (!on) continue;  // wave-uniform
            const HeRec Rh = he[3 * fs + k];
            const int t = Rh.twin, g = t / 3, m = t % 3;
            const HeRec Rt = he[t];
            const double ex = (P[(k + 1) % 3][0] - P[k][0]) / Rh.L, ey = (P[(k + 1) % 3][1] - P[k][1]) / Rh.L;
            const double c = -ex, s = -ey;
            const double ptx = Rh.L - (sb[(k + 1) % 3] * Rh.L + sb[(k + 2) % 3] * Rh.cx);
            int q = lane == 0 ? sd.fstart[g] : 0, q1 = lane == 0 ? sd.fstart[g + 1] : 0;
            while (__ballot(q < q1)) {
                bool ok = false;
                int j = 0;
                double d = 0, tx = 0, ty = 0;
                if (q < q1) {
                    j = sd.forder[q];
                    if (j != src) {
                        const double *b = sd.bary + 3 * (int64_t)j;
                        const double qx = b[(m + 1) % 3] * Rt.L + b[(m + 2) % 3] * Rt.cx;
                        const double qy = b[(m + 2) % 3] * Rt.cy;
                        double dx = qx - ptx, dy = qy;
                        d = sqrt(dx * dx + dy * dy);
                        if (d > 0) {
                            dx /= d;
                            dy /= d;
                            tx = c * dx - s * dy;
                            ty = s * dx + c * dy;
                        }
                        ok = true;
                    }
                    ++q;
                }
                target_update(L, td, tt, C, ok, j, d, tx, ty, INFINITY);
            }
            const double dx = Rt.cx - ptx, dy = Rt.cy;
            const double d = sqrt(dx * dx + dy * dy);
            const int opp = Rt.opp_flags >> 1;
            if (lane == 0) vdist_min(Dv, opp, d);
            const int eo = lane == 0 ? M.pidx[opp] : -1;
            bend_update(G, L.B, C.rc, eo >= 0, eo, d, (c * dx - s * dy) / d, (s * dx + c * dy) / d, INFINITY);
        }
        S.push(want, false, w, overflow);
        S.push(wantA, ka >= T, wa, overflow);
        S.push(wantB, kb >= T, wb, overflow);
    }

    // ---- propagation, round by round
    bool have = false;
    Win<R> w;
    unsigned long long nwin = 0;
    int pruned = 0, depth = 0;
    for (;;) {
        if (__ballot(overflow)) overflow = true;
        if (overflow) break;
        depth = max(depth, S.lsp + S.gsp + S.dsp);
        bool busy = S.refill(have, w);
        if (!busy && L.B.npend > 0) {
            launch_roots(a, sd, L, G, td, tt, Dv, C, S, T, src, st);
            busy = S.refill(have, w);
        }
        if (!busy) {
            if (S.dsp == 0 && L.B.npend == 0) break;
            // next round; once every target is reached, bound the keys
            S.next_round();
            T += C.bucket;
            if (L.unfound == 0) {
                __syncthreads();  // every lane's target stores are visible
                double mx = 0.0;
                for (int j = lane; j < n; j += kWave)
                    if (j != src) mx = fmax(mx, td[j].x);
                for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
                if (lane == 0) L.maxb = fmin(L.maxb, mx * (1.0 + C.tie_rel) + 1e-12 * mx);
            }
            __syncthreads();
            continue;
        }
        nwin += (unsigned long long)__popcll(__ballot(have));
        if (nwin > (unsigned long long)a.gp.max_windows) {
            overflow = true;
            break;
        }
        // stale: from an earlier launch of its root, or a new launch is due
        if (have && w.root >= 0 && bend_stale(G.rD[w.root], G.rL[w.root], w, C.rc)) {
            have = false;
            ++st.stale;
        }
        He<R> H;
        double txc = 0.0;
        int f = -1, k = 0, vA = 0, vB = 0;
        if (have) {
            f = w.he / 3;
            k = w.he % 3;
            H = load_he(M, w.he, R(0));
            vA = he[w.he].tail;
            vB = he[w.he].head;
            txc = (double)w.px + ((double)H.cx - (double)w.px) * (-(double)w.py) / ((double)H.cy - (double)w.py);
        }
        // vertices of the face reached through this window: the table's
        // values are read first (independent loads) and combined with this
        // window's own paths, which then go to the table
        double DA = INFINITY, DB = INFINITY, DC = INFINITY;
        bool cin = false;
        double dcv = 0.0;
        if (have) {
            DA = Dv[vA];
            DB = Dv[vB];
            DC = Dv[H.opp];
            const double px = w.px, py = w.py, sg = w.sg;
            if ((double)w.b0 <= 0.0) {
                const double d = sg + sqrt(px * px + py * py);
                if (d < DA) {
                    DA = d;
                    vdist_min(Dv, vA, d);
                }
            }
            if ((double)w.b1 >= (double)H.L) {
                const double d = sg + sqrt((H.L - px) * (H.L - px) + py * py);
                if (d < DB) {
                    DB = d;
                    vdist_min(Dv, vB, d);
                }
            }
            const double sl = C.tol * (double)H.L;
            cin = txc >= (double)w.b0 - sl && txc <= (double)w.b1 + sl;
            if (cin) {
                const double dx = (double)H.cx - px, dy = (double)H.cy - py;
                dcv = sg + sqrt(dx * dx + dy * dy);
                if (dcv < DC) {
                    DC = dcv;
                    vdist_min(Dv, H.opp, dcv);
                }
            }
        }
        query_face(sd, L, G, td, tt, C, have, src, f, k, H, w);
        // third vertex as a bend vertex
        {
            bool ok = have && H.pseudo && cin;
            double tx = 0, ty = 0, alt = INFINITY;
            if (ok) {
                if (w.root < 0) {
                    R dx = H.cx - w.px, dy = H.cy - w.py;
                    const R l = sqrt(dx * dx + dy * dy);
                    tx = (double)(w.c * (dx / l) - w.s * (dy / l));
                    ty = (double)(w.s * (dx / l) + w.c * (dy / l));
                } else {
                    tx = G.rtx[w.root];
                    ty = G.rty[w.root];
                    alt = G.rD2[w.root] + (dcv - (double)w.sg);
                }
            }
            const int eo = ok ? M.pidx[H.opp] : -1;
            bend_update(G, L.B, C.rc, ok, eo, dcv, tx, ty, alt);
        }
        // children, trimmed against the vertex paths and bounded by maxb
        Win<R> cl, cr;
        bool hl = false, hr = false;
        double kl = 0, kr = 0;
        if (have) {
            const double maxb = L.maxb;
            if (H.tp >= 0 && (double)w.b0 < txc) {
                double x0, x1;
                child_left(H, w, txc, false, x0, x1);
                make_left(H, w, x0, x1, cl);
                // edge A -> C: S = A, E = C; the face's third vertex B sits at
                // (ex L, -ey L) in the child frame
                double f0, f1;
                if (x1 - x0 > 1e-12 * (double)H.Lp &&
                    vertex_trim(cl.px, cl.py, cl.sg, H.Lp, DA, DC, C.dom_rel, x0, x1, f0, f1) &&
                    !opposite_dominates((double)H.ex * (double)H.L, -(double)H.ey * (double)H.L, DB, C.dom_rel, x0,
                                        x1, f0, f1)) {
                    cl.b0 = (R)x0;
                    cl.b1 = (R)x1;
                    kl = child_key(cl, f0, f1);
                    hl = kl < maxb;
                }
                if (!hl) ++pruned;
            }
            if (H.tn >= 0 && (double)w.b1 > txc) {
                double x0, x1;
                child_right(H, w, txc, false, x0, x1);
                make_right(H, w, x0, x1, cr);
                // edge C -> B: S = C, E = B; the third vertex A sits at
                // (-ux cx - uy cy, uy cx - ux cy) in the child frame
                const double ux = H.ux, uy = H.uy, hcx = H.cx, hcy = H.cy;
                double f0, f1;
                if (x1 - x0 > 1e-12 * (double)H.Ln &&
                    vertex_trim(cr.px, cr.py, cr.sg, H.Ln, DC, DB, C.dom_rel, x0, x1, f0, f1) &&
                    !opposite_dominates(-ux * hcx - uy * hcy, uy * hcx - ux * hcy, DA, C.dom_rel, x0, x1, f0, f1)) {
                    cr.b0 = (R)x0;
                    cr.b1 = (R)x1;
                    kr = child_key(cr, f0, f1);
                    hr = kr < maxb;
                }
                if (!hr) ++pruned;
            }
        }
        // children of the next round wait; of the two of this round, the lane keeps one
        const bool keep_l = hl && kl < T, keep_r = hr && kr < T;
        S.push(hl && !(keep_l), kl >= T, cl, overflow);
        S.push(hr && (keep_l || !keep_r), kr >= T, cr, overflow);
        if (have) {
            if (keep_l) w = cl;
            else if (keep_r) w = cr;
            else have = false;
        }
    }

    // ---- results: row src, entry j for target j
    const int32_t *Tt = M.T;
    const double *p0 = M.V + 3 * (int64_t)Tt[3 * fs], *p1 = M.V + 3 * (int64_t)Tt[3 * fs + 1];
    const double *nn = M.fnrm + 3 * (int64_t)fs;
    double ex3[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    const double el = sqrt(ex3[0] * ex3[0] + ex3[1] * ex3[1] + ex3[2] * ex3[2]);
    ex3[0] /= el;
    ex3[1] /= el;
    ex3[2] /= el;
    const double ey3[3] = {nn[1] * ex3[2] - nn[2] * ex3[1], nn[2] * ex3[0] - nn[0] * ex3[2],
                           nn[0] * ex3[1] - nn[1] * ex3[0]};
    const bool ovf = __ballot(overflow) != 0;
    const int64_t c0 = (int64_t)src * sd.cap;
    bool near_cut = false;
    __syncthreads();  // every lane's tangent stores are visible
    for (int j = lane; j < n; j += kWave) {
        const int64_t o = c0 + j;
        const double2 dd = td[j];
        double d = dd.x;
        uint8_t fl = guard ? GSIM_PAIR_GUARD_BIT : 0;
        if (j == src) d = INFINITY;
        else if (ovf) d = NAN;
        if (j != src && dd.y - d <= C.tie_rel * d) fl |= GSIM_PAIR_TIE_BIT;
        if (d == 0.0) fl |= GSIM_PAIR_ZERO_BIT;
        near_cut |= C.cutoff < INFINITY && fabs(d - C.cutoff) <= a.gp.guard_rel * C.cutoff;
        sd.cdist[o] = d;
        sd.cflags[o] = fl;
        const double2 t = tt[j];
        for (int qd = 0; qd < 3; ++qd) sd.ctan[3 * o + qd] = t.x * ex3[qd] + t.y * ey3[qd];
    }
    if (sd.prof && lane == 0) {
        long long *qp = sd.prof + 8 * (int64_t)src;
        qp[2] += (long long)nwin;
    }
    st.windows += nwin;
    st.pruned += pruned;
    st.overflow |= ovf;
    st.depth = max(st.depth, depth);
    bend_reset(G, L.B);
    return fp32 && !ovf && __ballot(near_cut) != 0;
}

template <bool kMixed, int kStk>
__global__ __launch_bounds__(kWave) void k_geodesic_all(AllArgs a) {
    __shared__ AllLds L;
    __shared__ alignas(16) unsigned char stk[kStk];
    double2 *td = a.ttab + (size_t)blockIdx.x * 2 * a.tcap, *tt = td + a.tcap;
    const int lane = lane_id();
    const int total = a.bi.begin[a.bi.nsurf];
    int chunk = blockIdx.x % kChunks, chunks_left = kChunks;
    SrcStats st;
    st.windows = st.launches = st.stale = st.guards = 0;
    st.pruned = 0;
    st.depth = 0;
    st.overflow = false;
    unsigned long long c_limited = 0;
    int next = 0, left = 0;
    for (;;) {
        if (left == 0) {
            while (chunks_left > 0) {
                const int lo = (int)(((int64_t)total * chunk) / kChunks);
                const int hi = (int)(((int64_t)total * (chunk + 1)) / kChunks);
                int t = 0;
                if (lane == 0) t = atomicAdd(&a.work[chunk * kWorkStride], a.grab);
                t = __shfl(t, 0);
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
        const int src = idx - a.bi.begin[si];
        if (lane == 0) sd.cand_cnt[src] = sd.n;
        st.overflow = false;
        bool again = !kMixed;
        if (kMixed) again = run_all<float>(a, sd, L, td, tt, stk, kStk, src, blockIdx.x, false, st);
        if (again) {
            // FP64 (the plain path, or the recompute of an FP32 source whose
            // results come too close to the cutoff to decide in FP32)
            run_all<double>(a, sd, L, td, tt, stk, kStk, src, blockIdx.x, kMixed, st);
            st.guards += kMixed ? 1 : 0;
        }
        if (st.overflow) ++c_limited;
    }
    unsigned long long pr = (unsigned long long)st.pruned, sl = st.stale;
    for (int o = 32; o > 0; o >>= 1) {
        pr += __shfl_xor(pr, o);
        sl += __shfl_xor(sl, o);
    }
    if (lane == 0) {
        atomicAdd(&a.ctr->windows, st.windows);
        atomicAdd(&a.ctr->pruned, pr);
        atomicAdd(&a.ctr->launches, st.launches);
        atomicAdd(&a.ctr->stale, sl);
        atomicAdd(&a.ctr->guards, st.guards);
        atomicAdd(&a.ctr->limited, c_limited);
        atomicMax(&a.ctr->max_depth, (unsigned long long)st.depth);
    }
}

template <bool kMixed>
const void *kernel_of(int kb) {
    if (kb <= 4) return (const void *)&k_geodesic_all<kMixed, 4096>;
    if (kb <= 8) return (const void *)&k_geodesic_all<kMixed, 8192>;
    return (const void *)&k_geodesic_all<kMixed, 16384>;
}

template <bool kMixed>
void launch_variant(int kb, int nslots, const AllArgs &a, hipStream_t s) {
    if (kb <= 4) hipLaunchKernelGGL((k_geodesic_all<kMixed, 4096>), dim3(nslots), dim3(kWave), 0, s, a);
    else if (kb <= 8) hipLaunchKernelGGL((k_geodesic_all<kMixed, 8192>), dim3(nslots), dim3(kWave), 0, s, a);
    else hipLaunchKernelGGL((k_geodesic_all<kMixed, 16384>), dim3(nslots), dim3(kWave), 0, s, a);
}

}  // namespace

hipError_t launch_geodesic_all(const SurfDesc *desc, const BatchIdx &bi, const GeoParams &gp, const GeoShape &shape,
                               char *stack_mem, double *vdist, int64_t vstride, char *roots, int64_t rstride,
                               int rcap, double2 *ttab, int tcap, int32_t *work_ctr, Counters *ctr, bool fp32,
                               hipStream_t s) {
    AllArgs a;
    a.sd = desc;
    a.bi = bi;
    a.gp = gp;
    a.stack = stack_mem;
    a.vdist = vdist;
    a.vstride = vstride;
    a.roots = roots;
    a.rstride = rstride;
    a.rcap = rcap;
    a.work = work_ctr;
    a.ctr = ctr;
    a.tcap = tcap;
    a.grab = shape.grab < 1 ? 1 : shape.grab;
    if (shape.nslots < 1 || bi.begin[bi.nsurf] < 1) return hipSuccess;
    a.ttab = ttab;
    if (fp32) launch_variant<true>(shape.lds_stack_kb, shape.nslots, a, s);
    else launch_variant<false>(shape.lds_stack_kb, shape.nslots, a, s);
    return hipGetLastError();
}

int geodesic_all_blocks_per_cu(int lds_stack_kb, bool fp32) {
    int nb = 0;
    const void *f = fp32 ? kernel_of<true>(lds_stack_kb) : kernel_of<false>(lds_stack_kb);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kWave, 0) != hipSuccess)
        return 0;
    return nb;
}

}  // namespace gsim
