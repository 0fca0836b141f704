// In-surface Voronoi neighbours of the particles (arXiv 2404.19751, Sec. 5:
// the restricted Euclidean Voronoi diagram from which coordination numbers
// and crystalline defects are read). The cell of particle i is the set of
// surface points no farther (3D distance) from x_i than from any other
// particle; two particles are neighbours when their cells share a boundary
// of positive length.
//
// Mapping: one wave64 per mesh face. The wave finds the particles that can
// be nearest somewhere on the face (those within the face's distance bound,
// from rings of a particle cell grid), one lane per such candidate; each
// lane clips the face, in the face's own 2D frame, by the bisector
// half-planes of the other candidates (Sutherland-Hodgman in LDS, every edge
// labelled with the particle whose bisector made it). Every clipped edge
// longer than the tolerance is a shared cell boundary: its two particles
// are marked in an n x n adjacency bitset (64-bit atomic OR). A second pair
// of kernels turns the bitset into a CSR sorted by neighbour.
#include <cmath>

#include "gsim_internal.h"

namespace gsim {
namespace {

constexpr int kWave = 64;
constexpr int kCand = 64;  // candidates per face: one lane each
constexpr int kPoly = 16;  // vertices of one clipped cell

struct VorArgs {
    DevMesh m;
    int n;
    const double *xyz;
    const int32_t *cell_start, *order;
    int dims[3];
    double lo[3], cell;
    unsigned long long *bits;  // [n][words]
    int64_t words;
    double tol;
    int32_t *err;  // [0] faces over the candidate limit, [1] cells over the vertex limit
};

struct V2 {
    double u, v;
};

// Squared distance from the 2D point q to the triangle (0,0), (b,0), c:
// zero inside, else to the nearest edge.
__device__ inline double tri2_dist2(V2 q, double bx, V2 c) {
    const V2 P[3] = {{0.0, 0.0}, {bx, 0.0}, c};
    // inside when on the left of all three counter-clockwise edges
    bool inside = true;
    double best = INFINITY;
    for (int k = 0; k < 3; ++k) {
        const V2 a = P[k], b = P[(k + 1) % 3];
        const double ex = b.u - a.u, ey = b.v - a.v;
        const double qx = q.u - a.u, qy = q.v - a.v;
        if (ex * qy - ey * qx < 0.0) inside = false;
        double t = (qx * ex + qy * ey) / (ex * ex + ey * ey);
        t = fmin(fmax(t, 0.0), 1.0);
        const double dx = qx - t * ex, dy = qy - t * ey;
        best = fmin(best, dx * dx + dy * dy);
    }
    return inside ? 0.0 : best;
}

__global__ __launch_bounds__(kWave) void k_voronoi_faces(VorArgs a) {
    __shared__ int32_t cid[kCand];
    __shared__ double cxyz[kCand][3];
    __shared__ double pu[2][kCand][kPoly], pv[2][kCand][kPoly];
    __shared__ int32_t plab[2][kCand][kPoly];
    __shared__ int32_t ncand;
    const int lane = threadIdx.x;
    const int f = blockIdx.x;
    const double *fp = a.m.fpos + 18 * (int64_t)f;
    const double A[3] = {fp[0], fp[1], fp[2]}, B[3] = {fp[3], fp[4], fp[5]}, Cv[3] = {fp[6], fp[7], fp[8]};
    // face frame: origin A, ex along AB, ey in the plane towards C, nz normal
    double ex[3], ey[3], nz[3];
    const double lab = sqrt((B[0] - A[0]) * (B[0] - A[0]) + (B[1] - A[1]) * (B[1] - A[1]) +
                            (B[2] - A[2]) * (B[2] - A[2]));
    for (int d = 0; d < 3; ++d) ex[d] = (B[d] - A[d]) / lab;
    const double ac[3] = {Cv[0] - A[0], Cv[1] - A[1], Cv[2] - A[2]};
    nz[0] = ex[1] * ac[2] - ex[2] * ac[1];
    nz[1] = ex[2] * ac[0] - ex[0] * ac[2];
    nz[2] = ex[0] * ac[1] - ex[1] * ac[0];
    const double nl = sqrt(nz[0] * nz[0] + nz[1] * nz[1] + nz[2] * nz[2]);
    for (int d = 0; d < 3; ++d) nz[d] /= nl;
    ey[0] = nz[1] * ex[2] - nz[2] * ex[1];
    ey[1] = nz[2] * ex[0] - nz[0] * ex[2];
    ey[2] = nz[0] * ex[1] - nz[1] * ex[0];
    const V2 C2 = {ac[0] * ex[0] + ac[1] * ex[1] + ac[2] * ex[2], ac[0] * ey[0] + ac[1] * ey[1] + ac[2] * ey[2]};
    double cen[3], rT = 0.0;
    for (int d = 0; d < 3; ++d) cen[d] = (A[d] + B[d] + Cv[d]) / 3.0;
    for (const double *P : {A, B, Cv}) {
        const double dx = P[0] - cen[0], dy = P[1] - cen[1], dz = P[2] - cen[2];
        rT = fmax(rT, sqrt(dx * dx + dy * dy + dz * dz));
    }
    int cc[3];
    for (int d = 0; d < 3; ++d) {
        const int q = (int)floor((cen[d] - a.lo[d]) / a.cell);
        cc[d] = q < 0 ? 0 : (q >= a.dims[d] ? a.dims[d] - 1 : q);
    }
    const int rmax_grid = max(a.dims[0], max(a.dims[1], a.dims[2]));

    // 1. distance bound: the smallest, over particles, farthest-vertex
    //    distance, from rings of cells around the centroid's cell (a
    //    particle beyond ring r is at least r cells from the centroid, and
    //    its farthest vertex no nearer than the centroid)
    double m2 = INFINITY;
    for (int r = 0; r <= rmax_grid; ++r) {
        const int w = 2 * r + 1;
        double lm = INFINITY;
        for (int q = lane; q < w * w * w; q += kWave) {
            const int dx = q % w - r, dy = (q / w) % w - r, dz = q / (w * w) - r;
            if (max(abs(dx), max(abs(dy), abs(dz))) != r) continue;
            const int x = cc[0] + dx, y = cc[1] + dy, z = cc[2] + dz;
            if (x < 0 || y < 0 || z < 0 || x >= a.dims[0] || y >= a.dims[1] || z >= a.dims[2]) continue;
            const int lin = (z * a.dims[1] + y) * a.dims[0] + x;
            for (int p = a.cell_start[lin]; p < a.cell_start[lin + 1]; ++p) {
                const double *xp = a.xyz + 3 * (int64_t)a.order[p];
                double far2 = 0.0;
                for (const double *P : {A, B, Cv}) {
                    const double ux = P[0] - xp[0], uy = P[1] - xp[1], uz = P[2] - xp[2];
                    far2 = fmax(far2, ux * ux + uy * uy + uz * uz);
                }
                lm = fmin(lm, far2);
            }
        }
        for (int o = 32; o > 0; o >>= 1) lm = fmin(lm, __shfl_xor(lm, o));
        m2 = fmin(m2, lm);
        if (m2 < INFINITY && (double)r * a.cell >= sqrt(m2)) break;
    }

    // 2. candidates: every particle whose distance to the face is within the
    //    bound (a particle can be nearest somewhere on the face only then)
    if (lane == 0) ncand = 0;
    __syncthreads();
    const double bound2 = m2 * (1.0 + 1e-9);
    const double reach = sqrt(bound2) + rT;
    const int rc = min((int)ceil(reach / a.cell) + 1, rmax_grid);
    const int wc = 2 * rc + 1;
    for (int q = lane; q < wc * wc * wc; q += kWave) {
        const int x = cc[0] + q % wc - rc, y = cc[1] + (q / wc) % wc - rc, z = cc[2] + q / (wc * wc) - rc;
        if (x < 0 || y < 0 || z < 0 || x >= a.dims[0] || y >= a.dims[1] || z >= a.dims[2]) continue;
        const int lin = (z * a.dims[1] + y) * a.dims[0] + x;
        for (int p = a.cell_start[lin]; p < a.cell_start[lin + 1]; ++p) {
            const int j = a.order[p];
            const double *xp = a.xyz + 3 * (int64_t)j;
            const double r0 = xp[0] - A[0], r1 = xp[1] - A[1], r2 = xp[2] - A[2];
            const double h = r0 * nz[0] + r1 * nz[1] + r2 * nz[2];
            const V2 qp = {r0 * ex[0] + r1 * ex[1] + r2 * ex[2], r0 * ey[0] + r1 * ey[1] + r2 * ey[2]};
            if (h * h + tri2_dist2(qp, lab, C2) <= bound2) {
                const int s = atomicAdd(&ncand, 1);
                if (s < kCand) {
                    cid[s] = j;
                    cxyz[s][0] = xp[0];
                    cxyz[s][1] = xp[1];
                    cxyz[s][2] = xp[2];
                }
            }
        }
    }
    __syncthreads();
    const int K = ncand;
    if (K > kCand) {
        if (lane == 0) atomicAdd(&a.err[0], 1);
        return;
    }

    // 3. lane i clips the face by the bisector half-planes of the others:
    //    |x - x_i|^2 <= |x - x_k|^2  <=>  2 (x_k - x_i).x <= |x_k|^2 - |x_i|^2
    bool over = false;
    if (lane < K) {
        int cur = 0, nv = 3;
        pu[0][lane][0] = 0.0;  pv[0][lane][0] = 0.0;  plab[0][lane][0] = -1;
        pu[0][lane][1] = lab;  pv[0][lane][1] = 0.0;  plab[0][lane][1] = -1;
        pu[0][lane][2] = C2.u; pv[0][lane][2] = C2.v; plab[0][lane][2] = -1;
        const double *xi = cxyz[lane];
        for (int k = 0; k < K && nv > 0; ++k) {
            if (k == lane) continue;
            const double *xk = cxyz[k];
            const double w0 = 2.0 * (xk[0] - xi[0]), w1 = 2.0 * (xk[1] - xi[1]), w2 = 2.0 * (xk[2] - xi[2]);
            // the half-plane in face coordinates: au u + av v <= c0
            const double au = w0 * ex[0] + w1 * ex[1] + w2 * ex[2];
            const double av = w0 * ey[0] + w1 * ey[1] + w2 * ey[2];
            const double c0 = (xk[0] * xk[0] + xk[1] * xk[1] + xk[2] * xk[2]) -
                              (xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]) - (w0 * A[0] + w1 * A[1] + w2 * A[2]);
            const int nxt = cur ^ 1;
            int no = 0;
            for (int j = 0; j < nv; ++j) {
                const int j2 = j + 1 == nv ? 0 : j + 1;
                const double u0 = pu[cur][lane][j], v0 = pv[cur][lane][j];
                const double u1 = pu[cur][lane][j2], v1 = pv[cur][lane][j2];
                const double s0 = au * u0 + av * v0 - c0, s1 = au * u1 + av * v1 - c0;
                const int lb = plab[cur][lane][j];
                if (s0 <= 0.0) {
                    if (no < kPoly) {
                        pu[nxt][lane][no] = u0;
                        pv[nxt][lane][no] = v0;
                        plab[nxt][lane][no] = lb;
                    }
                    ++no;
                    if (s1 > 0.0) {
                        // leaves the half-plane: the next edge lies on the bisector of k
                        const double t = s0 / (s0 - s1);
                        if (no < kPoly) {
                            pu[nxt][lane][no] = u0 + t * (u1 - u0);
                            pv[nxt][lane][no] = v0 + t * (v1 - v0);
                            plab[nxt][lane][no] = k;
                        }
                        ++no;
                    }
                } else if (s1 <= 0.0) {
                    // enters: the rest of edge j
                    const double t = s0 / (s0 - s1);
                    if (no < kPoly) {
                        pu[nxt][lane][no] = u0 + t * (u1 - u0);
                        pv[nxt][lane][no] = v0 + t * (v1 - v0);
                        plab[nxt][lane][no] = lb;
                    }
                    ++no;
                }
            }
            if (no > kPoly) {
                over = true;
                nv = 0;
                break;
            }
            nv = no;
            cur = nxt;
        }
        // 4. shared boundaries: every bisector edge longer than the tolerance
        const int i = cid[lane];
        for (int j = 0; j < nv; ++j) {
            const int lb = plab[cur][lane][j];
            if (lb < 0) continue;
            const int j2 = j + 1 == nv ? 0 : j + 1;
            const double du = pu[cur][lane][j2] - pu[cur][lane][j], dv = pv[cur][lane][j2] - pv[cur][lane][j];
            if (du * du + dv * dv > a.tol * a.tol) {
                const int k = cid[lb];
                atomicOr(&a.bits[(int64_t)i * a.words + (k >> 6)], 1ull << (k & 63));
                atomicOr(&a.bits[(int64_t)k * a.words + (i >> 6)], 1ull << (i & 63));
            }
        }
    }
    if (__ballot(over) && lane == 0) atomicAdd(&a.err[1], 1);
}

__global__ void k_voronoi_count(const unsigned long long *__restrict__ bits, int n, int64_t words,
                                int32_t *__restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    for (int64_t w = 0; w < words; ++w) c += __popcll(bits[(int64_t)i * words + w]);
    cnt[i] = c;
}

__global__ void k_voronoi_fill(const unsigned long long *__restrict__ bits, int n, int64_t words,
                               const int64_t *__restrict__ off, int32_t *__restrict__ nbr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t q = off[i];
    for (int64_t w = 0; w < words; ++w) {
        unsigned long long b = bits[(int64_t)i * words + w];
        while (b) {
            const int t = __ffsll(b) - 1;
            nbr[q++] = (int32_t)(w * 64 + t);
            b &= b - 1;
        }
    }
}

}  // namespace

hipError_t launch_voronoi_faces(const DevMesh &m, int n, const double *xyz, const int32_t *cell_start,
                                const int32_t *order, const int dims[3], const double lo[3], double cell,
                                unsigned long long *bits, int64_t words, double tol, int32_t *err, hipStream_t s) {
    if (m.nf <= 0 || n <= 0) return hipSuccess;
    VorArgs a;
    a.m = m;
    a.n = n;
    a.xyz = xyz;
    a.cell_start = cell_start;
    a.order = order;
    for (int d = 0; d < 3; ++d) {
        a.dims[d] = dims[d];
        a.lo[d] = lo[d];
    }
    a.cell = cell;
    a.bits = bits;
    a.words = words;
    a.tol = tol;
    a.err = err;
    hipLaunchKernelGGL(k_voronoi_faces, dim3(m.nf), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_voronoi_count(const unsigned long long *bits, int n, int64_t words, int32_t *cnt, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_voronoi_count, dim3((n + 255) / 256), dim3(256), 0, s, bits, n, words, cnt);
    return hipGetLastError();
}

hipError_t launch_voronoi_fill(const unsigned long long *bits, int n, int64_t words, const int64_t *off, int32_t *nbr,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_voronoi_fill, dim3((n + 255) / 256), dim3(256), 0, s, bits, n, words, off, nbr);
    return hipGetLastError();
}

}  // namespace gsim
