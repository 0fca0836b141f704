// Host-side mesh analysis for upload: half-edge twins, manifold and
// orientation checks, corner angles, pseudo-source vertices and the
// per-half-edge unfolding constants the kernels read.
//
// Pseudo-source vertices are the only places a shortest path may bend on a
// polyhedral surface: saddle vertices (corner-angle sum above 2 pi; the
// paper's spherical vertices, Sec. 3.2, are the opposite case) and boundary
// vertices. Vertices with sum >= 2 pi - 1e-9 are included so that nearly flat
// saddles are never missed.
#include <cmath>
#include <unordered_map>

#include "gsim_internal.h"

namespace gsim {

namespace {
inline uint64_t dkey(int32_t a, int32_t b) { return (uint64_t(uint32_t(a)) << 32) | uint32_t(b); }
struct V3 {
    double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 crs(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double nrm(V3 a) { return std::sqrt(dot(a, a)); }
}  // namespace

std::string build_host_mesh(int nv, const double *xyz, int nf, const int32_t *tri, HostMesh &M) {
    if (nv < 3 || nf < 1 || !xyz || !tri) return "empty mesh";
    for (size_t i = 0; i < 3 * (size_t)nv; ++i)
        if (!std::isfinite(xyz[i])) return "vertex coordinate not finite";
    const int ne = 3 * nf;
    M.nv = nv;
    M.nf = nf;
    M.V.assign(xyz, xyz + 3 * size_t(nv));
    M.T.assign(tri, tri + size_t(ne));
    for (int i = 0; i < ne; ++i)
        if (M.T[i] < 0 || M.T[i] >= nv) return "vertex index out of range";
    for (int f = 0; f < nf; ++f)
        if (M.T[3 * f] == M.T[3 * f + 1] || M.T[3 * f + 1] == M.T[3 * f + 2] || M.T[3 * f] == M.T[3 * f + 2])
            return "face with a repeated vertex";
    auto nxt = [](int h) { return h - h % 3 + (h % 3 + 1) % 3; };
    auto prv = [](int h) { return h - h % 3 + (h % 3 + 2) % 3; };
    auto P = [&](int v) { return V3{M.V[3 * size_t(v)], M.V[3 * size_t(v) + 1], M.V[3 * size_t(v) + 2]}; };

    // directed half-edge map; a directed edge seen twice means either a
    // non-manifold edge or two faces with opposite orientation
    std::unordered_map<uint64_t, int32_t> dir;
    dir.reserve(size_t(ne) * 2);
    for (int h = 0; h < ne; ++h) {
        auto r = dir.emplace(dkey(M.T[h], M.T[nxt(h)]), h);
        if (!r.second) return "non-manifold or inconsistently oriented edge";
    }
    M.twin.assign(ne, -1);
    M.n_boundary_edges = 0;
    for (int h = 0; h < ne; ++h) {
        auto it = dir.find(dkey(M.T[nxt(h)], M.T[h]));
        if (it != dir.end()) M.twin[h] = it->second;
        else M.n_boundary_edges++;
    }

    // corner angles, face normals, lengths
    M.corner.assign(ne, 0.0);
    M.theta.assign(nv, 0.0);
    M.fnrm.assign(3 * size_t(nf), 0.0);
    M.fpos.assign(18 * size_t(nf), 0.0);
    for (int f = 0; f < nf; ++f)
        for (int k = 0; k < 3; ++k) {
            V3 a = P(M.T[3 * f + k]), b = P(M.T[3 * f + (k + 1) % 3]);
            V3 u = sub(b, a);
            double l = nrm(u);
            double *q = M.fpos.data() + 18 * size_t(f);
            q[3 * k] = a.x;
            q[3 * k + 1] = a.y;
            q[3 * k + 2] = a.z;
            q[9 + 3 * k] = u.x / l;
            q[9 + 3 * k + 1] = u.y / l;
            q[9 + 3 * k + 2] = u.z / l;
        }
    double lsum = 0.0;
    int64_t lcnt = 0;
    M.min_edge = INFINITY;
    M.max_edge = 0.0;
    for (int f = 0; f < nf; ++f) {
        V3 n = crs(sub(P(M.T[3 * f + 1]), P(M.T[3 * f])), sub(P(M.T[3 * f + 2]), P(M.T[3 * f])));
        double a = nrm(n);
        if (!(a > 0.0)) return "degenerate face";
        M.fnrm[3 * f] = n.x / a;
        M.fnrm[3 * f + 1] = n.y / a;
        M.fnrm[3 * f + 2] = n.z / a;
        for (int k = 0; k < 3; ++k) {
            int h = 3 * f + k;
            V3 A = P(M.T[h]), B = P(M.T[nxt(h)]), C = P(M.T[prv(h)]);
            V3 u = sub(B, A), w = sub(C, A);
            double ang = std::atan2(nrm(crs(u, w)), dot(u, w));
            if (!(ang >= 1e-6)) return "face angle below 1e-6 rad";
            M.corner[h] = ang;
            M.theta[M.T[h]] += ang;
            double l = nrm(u);
            if (M.twin[h] < 0 || M.twin[h] > h) {
                lsum += l;
                lcnt++;
            }
            M.min_edge = std::fmin(M.min_edge, l);
            M.max_edge = std::fmax(M.max_edge, l);
        }
    }
    M.mean_edge = lsum / double(lcnt);

    // vertex fans in counter-clockwise order (next outgoing half-edge
    // around v is twin(prev(h))); an open fan starts at the half-edge with
    // no twin
    M.fan_off.assign(nv + 1, 0);
    for (int h = 0; h < ne; ++h) M.fan_off[M.T[h] + 1]++;
    for (int v = 0; v < nv; ++v) M.fan_off[v + 1] += M.fan_off[v];
    std::vector<int32_t> start(nv, -1);
    for (int h = 0; h < ne; ++h) {
        int v = M.T[h];
        if (start[v] < 0 || M.twin[h] < 0) start[v] = h;
    }
    M.fan.assign(ne, -1);
    M.vflag.assign(nv, 0);
    M.n_pseudo = 0;
    const double two_pi = 6.283185307179586476925286766559;
    for (int v = 0; v < nv; ++v) {
        int deg = M.fan_off[v + 1] - M.fan_off[v];
        if (deg == 0) continue;
        int h = start[v], got = 0;
        bool open = M.twin[h] < 0;
        while (got < deg) {
            M.fan[M.fan_off[v] + got++] = h;
            int nh = M.twin[prv(h)];
            if (nh < 0) {
                open = true;
                break;
            }
            if (nh == start[v]) break;
            h = nh;
        }
        if (got != deg) return "non-manifold vertex";
        uint8_t fl = 0;
        if (open) fl |= VF_BOUNDARY;
        if (open || M.theta[v] >= two_pi - 1e-9) fl |= VF_PSEUDO;
        M.vflag[v] = fl;
        if (fl & VF_PSEUDO) M.n_pseudo++;
    }
    // dense numbering of the pseudo-sources (the whole-mesh kernel's bend-vertex table)
    M.pidx.assign(nv, -1);
    M.pvert.clear();
    for (int v = 0; v < nv; ++v)
        if (M.vflag[v] & VF_PSEUDO) {
            M.pidx[v] = (int32_t)M.pvert.size();
            M.pvert.push_back(v);
        }
    if (M.pvert.empty()) M.pvert.push_back(-1);
    M.prec.assign(M.pvert.size(), PseudoRec{0.0, 0.0, 0.0, -1, 0, 0, 0});
    for (size_t e = 0; e < M.pvert.size(); ++e) {
        const int v = M.pvert[e];
        if (v < 0) continue;
        PseudoRec &r = M.prec[e];
        r.x = M.V[3 * size_t(v)];
        r.y = M.V[3 * size_t(v) + 1];
        r.z = M.V[3 * size_t(v) + 2];
        r.v = v;
        r.fan_beg = M.fan_off[v];
        r.fan_deg = M.fan_off[v + 1] - M.fan_off[v];
    }

    // unfolding records
    M.he.resize(ne);
    M.hef.resize(ne);
    for (int h = 0; h < ne; ++h) {
        V3 A = P(M.T[h]), B = P(M.T[nxt(h)]);
        int c = M.T[prv(h)];
        V3 C = P(c);
        V3 u = sub(B, A);
        double L = nrm(u);
        V3 e = {u.x / L, u.y / L, u.z / L};
        V3 w = sub(C, A);
        double cx = dot(w, e);
        double cy = nrm(crs(e, w));
        HeRec r;
        r.L = L;
        r.cx = cx;
        r.cy = cy;
        r.Lp = nrm(w);
        r.Ln = nrm(sub(C, B));
        // the same IEEE operations the kernels would do, so the values agree bit for bit
        r.ex = cx / r.Lp;
        r.ey = cy / r.Lp;
        r.ux = (L - cx) / r.Ln;
        r.uy = -cy / r.Ln;
        r.tn = M.twin[nxt(h)];
        r.tp = M.twin[prv(h)];
        r.opp_flags = (c << 1) | ((M.vflag[c] & VF_PSEUDO) ? 1 : 0);
        r.twin = M.twin[h];
        r.tail = M.T[h];
        r.head = M.T[nxt(h)];
        M.he[h] = r;
        HeRecF q;
        q.L = float(L);
        q.cx = float(cx);
        q.cy = float(cy);
        q.Lp = float(r.Lp);
        q.Ln = float(r.Ln);
        q.ex = q.cx / q.Lp;
        q.ey = q.cy / q.Lp;
        q.ux = (q.L - q.cx) / q.Ln;
        q.uy = -q.cy / q.Ln;
        q.tn = r.tn;
        q.tp = r.tp;
        q.opp_flags = r.opp_flags;
        M.hef[h] = q;
    }
    for (int d = 0; d < 3; ++d) {
        M.bbmin[d] = INFINITY;
        M.bbmax[d] = -INFINITY;
    }
    for (int v = 0; v < nv; ++v)
        for (int d = 0; d < 3; ++d) {
            M.bbmin[d] = std::fmin(M.bbmin[d], M.V[3 * size_t(v) + d]);
            M.bbmax[d] = std::fmax(M.bbmax[d], M.V[3 * size_t(v) + d]);
        }
    return std::string();
}

}  // namespace gsim
