// Streaming kernels around the geodesic pass: particle positions, the
// Euclidean cell-list prefilter, scans, CSR compaction, the force sum and
// the integrators. All are HBM-bound and written for coalesced access.
#include <cmath>

#include "gsim_internal.h"
#include "particle_ops.h"
#include "window.h"

namespace gsim {

namespace {
constexpr int kBlock = 256;
inline int nblocks(int64_t n, int b = kBlock) { return int((n + b - 1) / b); }

// ------------------------------------------------------------ positions
__global__ void k_xyz(const double *__restrict__ V, const int32_t *__restrict__ T, int n,
                      const int32_t *__restrict__ face, const double *__restrict__ bary, double *__restrict__ xyz) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int f = face[j];
    double b0 = bary[3 * j], b1 = bary[3 * j + 1], b2 = bary[3 * j + 2];
    const double *p0 = V + 3 * (int64_t)T[3 * f], *p1 = V + 3 * (int64_t)T[3 * f + 1],
                 *p2 = V + 3 * (int64_t)T[3 * f + 2];
    for (int d = 0; d < 3; ++d) xyz[3 * j + d] = b0 * p0[d] + b1 * p1[d] + b2 * p2[d];
}

__global__ void k_zero_i32(int32_t *p, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Empty bend-vertex tables: entry e of slot s gets infinite distances and
// is not queued (the tangent fields are written on insertion).
__global__ void k_bend_init(char *roots, int64_t rstride, int rcap, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int slot = (int)(i / rcap), e = (int)(i % rcap);
    const wnd::BendTable g = wnd::bend_table(roots, rstride, slot, rcap);
    g.rD[e] = INFINITY;
    g.rL[e] = INFINITY;
    g.rD2[e] = INFINITY;
    g.queued[e] = 0;
}

// ------------------------------------------------------------ scans
// Three-phase exclusive scan of int32 counts into int64 offsets:
// per-block totals, a single-block scan of the totals, then the block scan
// with its offset added. out[n] receives the grand total.
constexpr int kScanBlock = 1024;

__device__ inline int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t *total) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < blockDim.x; o <<= 1) {
        int64_t add = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t incl = sh[t];
    *total = sh[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_partials(const int32_t *__restrict__ in, int n, int64_t *__restrict__ part) {
    __shared__ int64_t sh[kScanBlock];
    int i = blockIdx.x * kScanBlock + threadIdx.x;
    int64_t v = i < n ? in[i] : 0;
    int64_t tot;
    block_excl_scan(v, sh, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void k_scan_partials_top(int64_t *part, int nb) {
    __shared__ int64_t sh[kScanBlock];
    int64_t carry = 0;
    for (int base = 0; base < nb; base += kScanBlock) {
        int i = base + threadIdx.x;
        int64_t v = i < nb ? part[i] : 0;
        int64_t tot;
        int64_t ex = block_excl_scan(v, sh, &tot);
        if (i < nb) part[i] = ex + carry;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) part[nb] = carry;
}

__global__ void k_scan_final(const int32_t *__restrict__ in, int n, const int64_t *__restrict__ part,
                             int64_t *__restrict__ out) {
    __shared__ int64_t sh[kScanBlock];
    int i = blockIdx.x * kScanBlock + threadIdx.x;
    int64_t v = i < n ? in[i] : 0;
    int64_t tot;
    int64_t ex = block_excl_scan(v, sh, &tot);
    if (i < n) out[i] = ex + part[blockIdx.x];
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = part[gridDim.x];
}

__global__ void k_i64_to_i32(const int64_t *in, int32_t *out, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) out[i] = int32_t(in[i]);
}

// ------------------------------------------------------------ prefilter
__device__ inline void cell_coords(const double *x, const PrefilterBufs &b, const double *bbmin, int c[3]) {
    for (int d = 0; d < 3; ++d) {
        int q = int(floor((x[d] - bbmin[d]) / b.cell));
        c[d] = q < 0 ? 0 : (q >= b.dims[d] ? b.dims[d] - 1 : q);
    }
}

struct BB {
    double lo[3];
};

// The cell counting sort of one surface whose grid is too fine for one
// workgroup's LDS, in four kernels: positions and cell counts (the first
// workgroup also starts the geodesic pass), the block totals of the counts,
// the cell starts (each block adds the totals of the blocks before it), and
// the scatter. The counts start from zeros and the scatter takes each back
// down to zero, so consecutive sorts need no clearing kernel between them.
__global__ void k_cell_count(const double *__restrict__ V, const int32_t *__restrict__ T, int n,
                             const int32_t *__restrict__ face, const double *__restrict__ bary, PrefilterBufs b,
                             BB bb, const SurfDesc *__restrict__ desc, int32_t *__restrict__ work, int advance) {
    if (work && blockIdx.x == 0) {
        // start of a pass: the geodesic kernel's work counters, and (in a
        // time step) the surface's step counter
        if (threadIdx.x < kWorkChunks) work[threadIdx.x * kWorkStride] = 0;
        if (advance && threadIdx.x == 0) *desc[0].step += 1;
    }
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int f = face[j];
    const double b0 = bary[3 * j], b1 = bary[3 * j + 1], b2 = bary[3 * j + 2];
    const double *p0 = V + 3 * (int64_t)T[3 * f], *p1 = V + 3 * (int64_t)T[3 * f + 1],
                 *p2 = V + 3 * (int64_t)T[3 * f + 2];
    double x[3];
    for (int d = 0; d < 3; ++d) {
        x[d] = b0 * p0[d] + b1 * p1[d] + b2 * p2[d];
        b.xyz[3 * j + d] = x[d];
    }
    int c[3];
    cell_coords(x, b, bb.lo, c);
    const int lin = (c[2] * b.dims[1] + c[1]) * b.dims[0] + c[0];
    b.cell_of[j] = lin;
    atomicAdd(&b.cell_fill[lin], 1);
}

__device__ inline int64_t block_sum(int64_t v, int64_t *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    int64_t t = 0;
    for (int k = 0; k < nw; ++k) t += sh[k];
    __syncthreads();
    return t;
}

__global__ void k_scan_final_i32(const int32_t *__restrict__ in, int n, const int64_t *__restrict__ part,
                                 int32_t *__restrict__ out) {
    __shared__ int64_t sh[kScanBlock];
    int64_t off = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += kScanBlock) off += part[k];
    off = block_sum(off, sh);
    const int i = blockIdx.x * kScanBlock + threadIdx.x;
    const int64_t v = i < n ? in[i] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan(v, sh, &tot);
    if (i < n) out[i] = (int32_t)(ex + off);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = (int32_t)(off + tot);
}

__global__ void k_bin_scatter(int n, PrefilterBufs b) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int lin = b.cell_of[j];
    int pos = b.cell_start[lin] + atomicSub(&b.cell_fill[lin], 1) - 1;
    b.order[pos] = j;
}

// Positions and the cell counting sort of one surface per workgroup: cell
// counts, their exclusive scan and the scatter all live in LDS. With
// `commit`, the particle state is first taken from the next-state arrays that
// the previous pass's fused update wrote (and copied into the current ones).
// Vertex positions come from the face record (one load after the face index);
// the scan runs within each wavefront by shuffles, then across the
// wavefronts through LDS (one barrier).
constexpr int kBinThreads = 1024;
constexpr int kBinWaves = kBinThreads / 64;
__global__ __launch_bounds__(kBinThreads) void k_bin_batch(const SurfDesc *__restrict__ desc,
                                                           int32_t *__restrict__ work, int advance, int commit) {
    __shared__ int32_t cnt[kSmallCells];
    __shared__ int32_t start[kSmallCells];
    __shared__ int32_t wsum[kBinWaves];
    const SurfDesc &sd = desc[blockIdx.x];
    // start of a pass: the geodesic kernel's work counters, and (in a time
    // step) the surface's step counter
    if (blockIdx.x == 0 && threadIdx.x < kWorkChunks) work[threadIdx.x * kWorkStride] = 0;
    if (advance && threadIdx.x == 0) *sd.step += 1;
    const double *__restrict__ fpos = sd.m.fpos;
    const int n = sd.n;
    const int t = threadIdx.x;
    const int lane = t & 63, wid = t >> 6;
    const int ncell = sd.dims[0] * sd.dims[1] * sd.dims[2];
    for (int c = t; c < ncell; c += kBinThreads) cnt[c] = 0;
    __syncthreads();
    int my_lin = 0;  // the cell of particle t (the first of the thread's particles)
    for (int j = t; j < n; j += kBinThreads) {
        const int32_t *face = commit ? sd.face_out : sd.face;
        const double *bary = commit ? sd.bary_out : sd.bary;
        const int f = face[j];
        const double b0 = bary[3 * j], b1 = bary[3 * j + 1], b2 = bary[3 * j + 2];
        if (commit) {
            sd.face[j] = f;
            sd.bary[3 * j] = b0;
            sd.bary[3 * j + 1] = b1;
            sd.bary[3 * j + 2] = b2;
            for (int q = 0; q < 3; ++q) sd.vel[3 * j + q] = sd.vel_out[3 * j + q];
        }
        const double *p0 = fpos + 18 * (int64_t)f, *p1 = p0 + 3, *p2 = p0 + 6;
        int c3[3];
        for (int d = 0; d < 3; ++d) {
            const double x = b0 * p0[d] + b1 * p1[d] + b2 * p2[d];
            sd.xyz[3 * j + d] = x;
            const int q = int(floor((x - sd.lo[d]) / sd.cell));
            c3[d] = q < 0 ? 0 : (q >= sd.dims[d] ? sd.dims[d] - 1 : q);
        }
        const int lin = (c3[2] * sd.dims[1] + c3[1]) * sd.dims[0] + c3[0];
        sd.cell_of[j] = lin;
        if (j == t) my_lin = lin;
        atomicAdd(&cnt[lin], 1);
    }
    __syncthreads();
    // exclusive scan: each thread owns a contiguous chunk of cells
    const int per = (ncell + kBinThreads - 1) / kBinThreads;
    const int c0 = t * per, c1 = min(c0 + per, ncell);
    int sum = 0;
    for (int c = c0; c < c1; ++c) sum += cnt[c];
    int incl = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int run = incl - sum;
    for (int w = 0; w < wid; ++w) run += wsum[w];
    for (int c = c0; c < c1; ++c) {
        start[c] = run;
        sd.cell_start[c] = run;
        run += cnt[c];
        cnt[c] = 0;
    }
    if (t == kBinThreads - 1) sd.cell_start[ncell] = run;
    __syncthreads();
    for (int j = t; j < n; j += kBinThreads) {
        const int lin = j == t ? my_lin : sd.cell_of[j];
        sd.order[start[lin] + atomicAdd(&cnt[lin], 1)] = j;
    }
}

__global__ void k_count_rows(int n, const int32_t *__restrict__ cnt, int cap, const double *__restrict__ dist,
                             double cutoff, int32_t *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0, m = min(cnt[i], cap);
    for (int s = 0; s < m; ++s) c += dist[(int64_t)i * cap + s] < cutoff;
    out[i] = c;
}

__global__ void k_compact_rows(int n, const int32_t *__restrict__ cnt, int cap, const int32_t *__restrict__ cand,
                               const double *__restrict__ dist, const double *__restrict__ tan,
                               const uint8_t *__restrict__ flags, double cutoff, const int64_t *__restrict__ off,
                               int32_t *__restrict__ nbr, double *__restrict__ od, double *__restrict__ ot,
                               uint8_t *__restrict__ of) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t q = off[i];
    int m = min(cnt[i], cap);
    for (int s = 0; s < m; ++s) {
        int64_t p = (int64_t)i * cap + s;
        if (!(dist[p] < cutoff)) continue;
        nbr[q] = cand[p];
        od[q] = dist[p];
        ot[3 * q] = tan[3 * p];
        ot[3 * q + 1] = tan[3 * p + 1];
        ot[3 * q + 2] = tan[3 * p + 2];
        of[q] = flags[p];
        ++q;
    }
}

// ------------------------------------------------------------ forces
__global__ void k_forces_rows(int n, const int32_t *__restrict__ cnt, int cap, const double *__restrict__ dist,
                              const double *__restrict__ tan, double cutoff, int kind, double k, double sigma,
                              double *__restrict__ F, double *__restrict__ Ei, unsigned long long *__restrict__ npairs,
                              uint8_t *__restrict__ pflags, unsigned long long *__restrict__ nonfinite) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int np = 0;
    bool bad = false;
    if (i < n) {
        double f[3], e;
        row_force(i, cnt, cap, dist, tan, cutoff, kind, k, sigma, f, e, np);
        F[3 * i] = f[0];
        F[3 * i + 1] = f[1];
        F[3 * i + 2] = f[2];
        Ei[i] = e;
        bad = !(isfinite(f[0]) && isfinite(f[1]) && isfinite(f[2]) && isfinite(e));
        if (pflags) pflags[i] = bad ? PF_NONFINITE : 0;
    }
    if (npairs) wave_atomic_add(npairs, (unsigned long long)np);
    if (nonfinite) wave_atomic_add(nonfinite, bad ? 1ull : 0ull);
}

// Euclidean candidates of every particle: the particles within the cutoff
// in the 27 cells around it (cells no smaller than the cutoff).
__global__ void k_count_candidates(int n, const double *__restrict__ xyz, const int32_t *__restrict__ cell_of,
                                   const int32_t *__restrict__ cell_start, const int32_t *__restrict__ order,
                                   int dx, int dy, int dz, double cut2, int32_t *__restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = xyz[3 * (int64_t)i], yi = xyz[3 * (int64_t)i + 1], zi = xyz[3 * (int64_t)i + 2];
    const int lin = cell_of[i];
    const int cx = lin % dx, cy = (lin / dx) % dy, cz = lin / (dx * dy);
    int m = 0;
    for (int z = max(cz - 1, 0); z <= min(cz + 1, dz - 1); ++z)
        for (int y = max(cy - 1, 0); y <= min(cy + 1, dy - 1); ++y)
            for (int x = max(cx - 1, 0); x <= min(cx + 1, dx - 1); ++x) {
                const int c = (z * dy + y) * dx + x;
                for (int q = cell_start[c]; q < cell_start[c + 1]; ++q) {
                    const int j = order[q];
                    const double ex = xyz[3 * (int64_t)j] - xi, ey = xyz[3 * (int64_t)j + 1] - yi,
                                 ez = xyz[3 * (int64_t)j + 2] - zi;
                    m += j != i && ex * ex + ey * ey + ez * ez < cut2;
                }
            }
    cnt[i] = m;
}

// A particle state is usable when every face index is in range and every
// barycentric triple lies in the face, sums to 1 and is not a vertex (the
// conditions the host path checks too), and every velocity is finite.
__global__ void k_validate_state(int nf, int n, const int32_t *__restrict__ face, const double *__restrict__ bary,
                                 const double *__restrict__ vel, int32_t *__restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int bf = 0, bb = 0, bv = 0;
    if (i < n) {
        const int f = face[i];
        bf = f < 0 || f >= nf;
        const double b0 = bary[3 * (int64_t)i], b1 = bary[3 * (int64_t)i + 1], b2 = bary[3 * (int64_t)i + 2];
        // written so that NaN fails every comparison
        const bool in01 = b0 >= 0.0 && b0 <= 1.0 && b1 >= 0.0 && b1 <= 1.0 && b2 >= 0.0 && b2 <= 1.0;
        const int zeros = (b0 == 0.0) + (b1 == 0.0) + (b2 == 0.0);
        bb = !(in01 && fabs(b0 + b1 + b2 - 1.0) <= 1e-9 && zeros < 2);
        if (vel) {
            const double *v = vel + 3 * (int64_t)i;
            bv = !(isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]));
        }
    }
    const unsigned long long mf = __ballot(bf), mb = __ballot(bb), mv = __ballot(bv);
    if ((threadIdx.x & 63) == 0) {
        if (mf) atomicAdd(&bad[0], __popcll(mf));
        if (mb) atomicAdd(&bad[1], __popcll(mb));
        if (mv) atomicAdd(&bad[2], __popcll(mv));
    }
}

// deterministic two-level sum
__global__ void k_sum_blocks(const double *__restrict__ x, int n, double *__restrict__ part) {
    __shared__ double sh[kBlock];
    int i = blockIdx.x * kBlock + threadIdx.x;
    sh[threadIdx.x] = i < n ? x[i] : 0.0;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void k_sum_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

// ------------------------------------------------------------ integrators
__global__ void k_integrate(int n, DevMesh m, const int32_t *__restrict__ face, const double *__restrict__ F, int kind,
                            double dt, double mob, double kT, double lam, uint64_t seed, uint64_t step,
                            double *__restrict__ D) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double f[3] = {F[3 * i], F[3 * i + 1], F[3 * i + 2]}, d[3];
    displacement(m, face[i], i, f, kind, dt, mob, kT, lam, seed, step, d);
    D[3 * i] = d[0];
    D[3 * i + 1] = d[1];
    D[3 * i + 2] = d[2];
}
// Start of a pass when the binning runs as several kernels: the work
// counters and (in a time step) the step counters.
__global__ void k_pass_begin(const SurfDesc *__restrict__ desc, int nsurf, int32_t *__restrict__ work, int advance) {
    const int t = threadIdx.x;
    if (t < kWorkChunks) work[t * kWorkStride] = 0;
    if (advance && t < nsurf) *desc[t].step += 1;
}
__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------ all-pairs
__global__ void k_face_count(int n, const int32_t *__restrict__ face, int32_t *__restrict__ counts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&counts[face[i]], 1);
}
__global__ void k_face_scatter(int n, const int32_t *__restrict__ face, const int32_t *__restrict__ fstart,
                               int32_t *__restrict__ counts, int32_t *__restrict__ forder) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int f = face[i];
        forder[fstart[f] + atomicAdd(&counts[f], 1)] = i;
    }
}
__global__ void k_identity_rows(int n, int cap, int32_t *__restrict__ cand_cnt, int32_t *__restrict__ cand) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * cap) return;
    const int i = (int)(t / cap), j = (int)(t % cap);
    cand[t] = j;
    if (j == 0) cand_cnt[i] = n;
}

// ------------------------------------------------------------ FIRE
// Force of every particle of the FIRE surfaces of a batch (kept for the
// update) and, per block of 256 particles of one surface, the partial sums
// of the power F.v and of |v|^2 and |F|^2 (fixed-order tree reduction).
__global__ __launch_bounds__(kFireBlock) void k_fire_partials(const SurfDesc *__restrict__ desc, BatchIdx blk,
                                                              double *__restrict__ partials,
                                                              unsigned long long *__restrict__ npairs) {
    __shared__ double sh[3][kFireBlock];
    const int b = blockIdx.x, t = threadIdx.x;
    const int si = batch_surface(blk, b);
    const SurfDesc &sd = desc[si];
    const int i = (b - blk.begin[si]) * kFireBlock + t;
    double p = 0.0, vv = 0.0, ff = 0.0;
    int np = 0;
    if (sd.ikind == 2 && i < sd.n) {
        double F[3], E;
        row_force(i, sd.cand_cnt, sd.cap, sd.cdist, sd.ctan, sd.cutoff, sd.pkind, sd.pk, sd.psigma, F, E, np);
        const double *v = sd.vel + 3 * (int64_t)i;
        for (int d = 0; d < 3; ++d) {
            sd.F[3 * (int64_t)i + d] = F[d];
            p += F[d] * v[d];
            vv += v[d] * v[d];
            ff += F[d] * F[d];
        }
    }
    wave_atomic_add(npairs, (unsigned long long)np);
    sh[0][t] = p;
    sh[1][t] = vv;
    sh[2][t] = ff;
    __syncthreads();
    for (int o = kFireBlock / 2; o > 0; o >>= 1) {
        if (t < o)
            for (int q = 0; q < 3; ++q) sh[q][t] += sh[q][t + o];
        __syncthreads();
    }
    if (t < 3) partials[3 * (int64_t)b + t] = sh[t][0];
}

// The FIRE control step of every FIRE surface (Bitzek et al., PRL 97,
// 170201 (2006)): with the power P = sum F.v of the current iteration,
// P > 0 mixes the velocities towards the force direction (v <- (1 - alpha) v
// + alpha |v| F/|F|) and, after more than n_min such iterations in a row,
// grows dt (up to dt_max) and shrinks alpha; P <= 0 stops the particles, cuts
// dt and resets alpha. The update kernel then applies v <- cv v + cf F,
// v += dt F, and walks dt v.
__global__ void k_fire_control(const SurfDesc *__restrict__ desc, BatchIdx blk, const double *__restrict__ partials) {
    const int si = blockIdx.x * blockDim.x + threadIdx.x;
    if (si >= blk.nsurf) return;
    const SurfDesc &sd = desc[si];
    if (sd.ikind != 2) return;
    double P = 0.0, vv = 0.0, ff = 0.0;
    for (int b = blk.begin[si]; b < blk.begin[si + 1]; ++b) {
        P += partials[3 * (int64_t)b];
        vv += partials[3 * (int64_t)b + 1];
        ff += partials[3 * (int64_t)b + 2];
    }
    FireState st = *sd.fire;
    if (!st.init) {
        st.dt = sd.dt;
        st.alpha = sd.alpha0;
        st.n_pos = 0;
        st.init = 1;
    }
    if (P > 0.0) {
        st.cv = 1.0 - st.alpha;
        st.cf = ff > 0.0 ? st.alpha * sqrt(vv) / sqrt(ff) : 0.0;
        if (!(ff > 0.0)) st.cv = 1.0;
        st.n_pos += 1;
        if (st.n_pos > sd.n_min) {
            st.dt = fmin(st.dt * sd.f_inc, sd.dt_max);
            st.alpha *= sd.f_alpha;
        }
    } else {
        st.cv = 0.0;
        st.cf = 0.0;
        st.dt *= sd.f_dec;
        st.alpha = sd.alpha0;
        st.n_pos = 0;
    }
    *sd.fire = st;
}

}  // namespace

// ------------------------------------------------------------ launchers
hipError_t launch_xyz(const DevMesh &m, int n, const int32_t *face, const double *bary, double *xyz, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_xyz, dim3(nblocks(n)), dim3(kBlock), 0, s, m.V, m.T, n, face, bary, xyz);
    return hipGetLastError();
}
hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_i32, dim3(nblocks(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_bend_init(char *roots, int nslots, int64_t rstride, int rcap, hipStream_t s) {
    const int64_t n = (int64_t)nslots * rcap;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bend_init, dim3(nblocks(n)), dim3(kBlock), 0, s, roots, rstride, rcap, n);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3(nblocks(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_scan_i32_to_i64(const int32_t *in, int64_t *out, int n, int64_t *scratch, hipStream_t s) {
    int nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_scan_partials, dim3(nb), dim3(kScanBlock), 0, s, in, n, scratch);
    hipLaunchKernelGGL(k_scan_partials_top, dim3(1), dim3(kScanBlock), 0, s, scratch, nb);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(kScanBlock), 0, s, in, n, scratch, out);
    return hipGetLastError();
}

hipError_t launch_cell_sort(const DevMesh &m, int n, const int32_t *face, const double *bary, PrefilterBufs &b,
                            int64_t *scratch, bool clear, const SurfDesc *desc, int32_t *work, bool advance,
                            hipStream_t s) {
    const int ncell = b.dims[0] * b.dims[1] * b.dims[2];
    BB bb;
    for (int d = 0; d < 3; ++d) bb.lo[d] = m.bbmin[d];
    hipError_t e;
    if (clear && (e = launch_zero_i32(b.cell_fill, ncell, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_count, dim3(std::max(1, nblocks(n))), dim3(kBlock), 0, s, m.V, m.T, n, face, bary, b,
                       bb, desc, work, advance ? 1 : 0);
    const int nb = std::max(1, (ncell + kScanBlock - 1) / kScanBlock);
    hipLaunchKernelGGL(k_scan_partials, dim3(nb), dim3(kScanBlock), 0, s, b.cell_fill, ncell, scratch);
    hipLaunchKernelGGL(k_scan_final_i32, dim3(nb), dim3(kScanBlock), 0, s, b.cell_fill, ncell, scratch,
                       b.cell_start);
    if (n > 0) hipLaunchKernelGGL(k_bin_scatter, dim3(nblocks(n)), dim3(kBlock), 0, s, n, b);
    return hipGetLastError();
}

hipError_t launch_bin_batch(const SurfDesc *desc, int nsurf, int32_t *work, bool advance, bool commit,
                            hipStream_t s) {
    if (nsurf <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin_batch, dim3(nsurf), dim3(kBinThreads), 0, s, desc, work, advance ? 1 : 0,
                       commit ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_pass_begin(const SurfDesc *desc, int nsurf, int32_t *work, bool advance, hipStream_t s) {
    hipLaunchKernelGGL(k_pass_begin, dim3(1), dim3(kMaxBatch), 0, s, desc, nsurf, work, advance ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(nblocks(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}
hipError_t launch_i64_to_i32(const int64_t *in, int32_t *out, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_i64_to_i32, dim3(nblocks(n + 1)), dim3(kBlock), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_count_rows(int n, const int32_t *cnt, int cap_c, const double *dist, double cutoff, int32_t *out,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_count_rows, dim3(nblocks(n)), dim3(kBlock), 0, s, n, cnt, cap_c, dist, cutoff, out);
    return hipGetLastError();
}
hipError_t launch_compact_rows(int n, const int32_t *cnt, int cap_c, const int32_t *cand, const double *dist,
                               const double *tan, const uint8_t *flags, double cutoff, const int64_t *off,
                               int32_t *nbr, double *odist, double *otan, uint8_t *oflags, hipStream_t s) {
    hipLaunchKernelGGL(k_compact_rows, dim3(nblocks(n)), dim3(kBlock), 0, s, n, cnt, cap_c, cand, dist, tan, flags,
                       cutoff, off, nbr, odist, otan, oflags);
    return hipGetLastError();
}
hipError_t launch_forces_rows(int n, const int32_t *cnt, int cap_c, const double *dist, const double *tan,
                              double cutoff, int kind, double k, double sigma, double *F, double *Ei,
                              unsigned long long *npairs, uint8_t *pflags, unsigned long long *nonfinite,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_forces_rows, dim3(nblocks(n)), dim3(kBlock), 0, s, n, cnt, cap_c, dist, tan, cutoff, kind, k,
                       sigma, F, Ei, npairs, pflags, nonfinite);
    return hipGetLastError();
}
hipError_t launch_count_candidates(int n, const PrefilterBufs &b, double cut2, int32_t *cnt, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_candidates, dim3(nblocks(n)), dim3(kBlock), 0, s, n, b.xyz, b.cell_of, b.cell_start,
                       b.order, b.dims[0], b.dims[1], b.dims[2], cut2, cnt);
    return hipGetLastError();
}
hipError_t launch_validate_state(int nf, int n, const int32_t *face, const double *bary, const double *vel,
                                 int32_t *bad, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate_state, dim3(nblocks(n)), dim3(kBlock), 0, s, nf, n, face, bary, vel, bad);
    return hipGetLastError();
}
hipError_t launch_sum(const double *x, int n, double *out, double *scratch, hipStream_t s) {
    int nb = nblocks(n);
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_sum_blocks, dim3(nb), dim3(kBlock), 0, s, x, n, scratch);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, scratch, nb, out);
    return hipGetLastError();
}
hipError_t launch_integrate(const DevMesh &m, int n, const int32_t *face, const double *F, int kind, double dt,
                            double mobility, double kT, double friction, uint64_t seed, uint64_t step, double *disp,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_integrate, dim3(nblocks(n)), dim3(kBlock), 0, s, n, m, face, F, kind, dt, mobility, kT,
                       friction, seed, step, disp);
    return hipGetLastError();
}

}  // namespace gsim

namespace gsim {
hipError_t launch_face_sort(const SurfDesc &d, int32_t *counts, int64_t *tmp64, int64_t *scan_scratch, hipStream_t s) {
    const int n = d.n, nf = d.m.nf;
    hipError_t e;
    if ((e = launch_zero_i32(counts, nf, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_face_count, dim3(nblocks(n)), dim3(kBlock), 0, s, n, d.face, counts);
    if ((e = launch_scan_i32_to_i64(counts, tmp64, nf, scan_scratch, s)) != hipSuccess) return e;
    if ((e = launch_i64_to_i32(tmp64, d.fstart, nf, s)) != hipSuccess) return e;
    if ((e = launch_zero_i32(counts, nf, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_face_scatter, dim3(nblocks(n)), dim3(kBlock), 0, s, n, d.face, d.fstart, counts, d.forder);
    return hipGetLastError();
}
hipError_t launch_identity_rows(int n, int cap, int32_t *cand_cnt, int32_t *cand, hipStream_t s) {
    hipLaunchKernelGGL(k_identity_rows, dim3(nblocks((int64_t)n * cap)), dim3(kBlock), 0, s, n, cap, cand_cnt, cand);
    return hipGetLastError();
}
hipError_t launch_fire_control(const SurfDesc *desc, const BatchIdx &blk, double *partials, Counters *ctr,
                               hipStream_t s) {
    const int nb = blk.begin[blk.nsurf];
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fire_partials, dim3(nb), dim3(kFireBlock), 0, s, desc, blk, partials, &ctr->nbr_pairs);
    hipLaunchKernelGGL(k_fire_control, dim3(1), dim3(kMaxBatch), 0, s, desc, blk, partials);
    return hipGetLastError();
}
}  // namespace gsim
