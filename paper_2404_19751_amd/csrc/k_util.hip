// Streaming kernels around the geodesic pass: particle positions, the
// Euclidean cell-list prefilter, scans, CSR compaction, the force sum and
// the integrators. All are HBM-bound and written for coalesced access.
#include <cmath>

#include "gsim_internal.h"

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

__global__ void k_bin_count(int n, PrefilterBufs b, BB bb) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int c[3];
    cell_coords(b.xyz + 3 * j, b, bb.lo, c);
    int lin = (c[2] * b.dims[1] + c[1]) * b.dims[0] + c[0];
    b.cell_of[j] = lin;
    atomicAdd(&b.cell_fill[lin], 1);
}

__global__ void k_bin_scatter(int n, PrefilterBufs b) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int lin = b.cell_of[j];
    int pos = b.cell_start[lin] + atomicAdd(&b.cell_fill[lin], 1);
    b.order[pos] = j;
}

// Candidate targets of each source: every particle whose Euclidean
// distance is below the cutoff (the paper's lower bound, Sec. 3.1), from the
// 27 cells around the source, kept sorted by particle index in a row of
// fixed capacity. cand_cnt holds the true count; a count above the capacity
// is reported through `overflow`.
__global__ void k_candidates_rows(int n, double cut2, PrefilterBufs b, int32_t *__restrict__ overflow) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = b.xyz[3 * i], yi = b.xyz[3 * i + 1], zi = b.xyz[3 * i + 2];
    int lin = b.cell_of[i];
    int cx = lin % b.dims[0], cy = (lin / b.dims[0]) % b.dims[1], cz = lin / (b.dims[0] * b.dims[1]);
    int cnt = 0;
    int32_t *row = b.cand + (int64_t)i * b.cap_c;
    for (int dz = -1; dz <= 1; ++dz) {
        int z = cz + dz;
        if (z < 0 || z >= b.dims[2]) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            int y = cy + dy;
            if (y < 0 || y >= b.dims[1]) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                int x = cx + dx;
                if (x < 0 || x >= b.dims[0]) continue;
                int c = (z * b.dims[1] + y) * b.dims[0] + x;
                for (int a = b.cell_start[c]; a < b.cell_start[c + 1]; ++a) {
                    int j = b.order[a];
                    if (j == i) continue;
                    double ex = b.xyz[3 * j] - xi, ey = b.xyz[3 * j + 1] - yi, ez = b.xyz[3 * j + 2] - zi;
                    if (ex * ex + ey * ey + ez * ez < cut2) {
                        if (cnt < b.cap_c) {
                            int p = cnt;
                            while (p > 0 && row[p - 1] > j) {
                                row[p] = row[p - 1];
                                --p;
                            }
                            row[p] = j;
                        }
                        ++cnt;
                    }
                }
            }
        }
    }
    b.cand_cnt[i] = cnt;
    if (cnt > b.cap_c) atomicAdd(overflow, 1);
}

// ------------------------------------------------------------ compaction
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
// F_i = sum_j U'(d_ij) t_ij and E_i = (1/2) sum_j U(d_ij), ascending j, over
// the pairs of the row closer than the cutoff.
__global__ void k_forces_rows(int n, const int32_t *__restrict__ cnt, int cap, const double *__restrict__ dist,
                              const double *__restrict__ tan, double cutoff, int kind, double k, double sigma,
                              double *__restrict__ F, double *__restrict__ Ei, unsigned long long *__restrict__ npairs) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
    int m = min(cnt[i], cap), np = 0;
    for (int s = 0; s < m; ++s) {
        int64_t p = (int64_t)i * cap + s;
        double d = dist[p];
        if (!(d < cutoff)) continue;
        ++np;
        if (!(d > 0.0)) continue;
        double U, dU;
        if (kind == 0) {  // harmonic
            if (d < sigma) {
                double x = 1.0 - d / sigma;
                U = 0.5 * k * x * x;
                dU = -(k / sigma) * x;
            } else {
                U = 0.0;
                dU = 0.0;
            }
        } else if (kind == 1) {  // coulomb
            U = k / d;
            dU = -k / (d * d);
        } else {  // gaussian
            U = k * exp(-d * d / (2.0 * sigma * sigma));
            dU = -(d / (sigma * sigma)) * U;
        }
        fx += dU * tan[3 * p];
        fy += dU * tan[3 * p + 1];
        fz += dU * tan[3 * p + 2];
        e += 0.5 * U;
    }
    F[3 * i] = fx;
    F[3 * i + 1] = fy;
    F[3 * i + 2] = fz;
    Ei[i] = e;
    if (npairs && np) atomicAdd(npairs, (unsigned long long)np);
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
// Philox4x32-10 (Salmon et al., SC'11): ten multiply-xor rounds, Weyl key
// schedule.
__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__global__ void k_integrate(int n, const double *__restrict__ V, const int32_t *__restrict__ T,
                            const double *__restrict__ fnrm, const int32_t *__restrict__ face,
                            const double *__restrict__ F, int kind, double dt, double mob, double kT, double lam,
                            uint64_t seed, uint64_t step, double *__restrict__ D) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (kind == 0) {
        double s = mob * dt;
        D[3 * i] = s * F[3 * i];
        D[3 * i + 1] = s * F[3 * i + 1];
        D[3 * i + 2] = s * F[3 * i + 2];
        return;
    }
    // Brownian: lam D = dt F + sqrt(2 kT lam dt) (eta1 ex + eta2 ey)
    uint32_t c[4] = {uint32_t(i), uint32_t(step), uint32_t(step >> 32), 0u};
    philox10(c, uint32_t(seed), uint32_t(seed >> 32));
    double u1 = (double(c[0] >> 5) * 67108864.0 + double(c[1] >> 6)) * (1.0 / 9007199254740992.0);
    double u2 = (double(c[2] >> 5) * 67108864.0 + double(c[3] >> 6)) * (1.0 / 9007199254740992.0);
    double r = sqrt(-2.0 * log(1.0 - u1));
    double sn, cs;
    sincos(2.0 * M_PI * u2, &sn, &cs);
    double e1 = r * cs, e2 = r * sn;
    int f = face[i];
    const double *p0 = V + 3 * (int64_t)T[3 * f], *p1 = V + 3 * (int64_t)T[3 * f + 1];
    double ex[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    double l = sqrt(ex[0] * ex[0] + ex[1] * ex[1] + ex[2] * ex[2]);
    ex[0] /= l;
    ex[1] /= l;
    ex[2] /= l;
    const double *nn = fnrm + 3 * (int64_t)f;
    double ey[3] = {nn[1] * ex[2] - nn[2] * ex[1], nn[2] * ex[0] - nn[0] * ex[2], nn[0] * ex[1] - nn[1] * ex[0]};
    double amp = sqrt(2.0 * kT * lam * dt) / lam, a = dt / lam;
    for (int d = 0; d < 3; ++d) D[3 * i + d] = a * F[3 * i + d] + amp * (e1 * ex[d] + e2 * ey[d]);
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

hipError_t launch_prefilter_bin(const DevMesh &m, int n, PrefilterBufs &b, hipStream_t s) {
    int ncell = b.dims[0] * b.dims[1] * b.dims[2];
    BB bb;
    for (int d = 0; d < 3; ++d) bb.lo[d] = m.bbmin[d];
    hipError_t e;
    if ((e = launch_zero_i32(b.cell_fill, ncell, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_count, dim3(nblocks(n)), dim3(kBlock), 0, s, n, b, bb);
    // cell_start = exclusive scan of cell_fill, computed through the int64 scan
    // into cand_off's storage is not possible (sizes differ); use a dedicated pass
    return hipGetLastError();
}

hipError_t launch_prefilter_rows(int n, double cutoff, PrefilterBufs &b, int32_t *overflow, hipStream_t s) {
    double c2 = cutoff * cutoff * (1.0 + 1e-12);
    hipLaunchKernelGGL(k_candidates_rows, dim3(nblocks(n, 64)), dim3(64), 0, s, n, c2, b, overflow);
    return hipGetLastError();
}
hipError_t launch_bin_scatter(int n, PrefilterBufs &b, hipStream_t s) {
    hipLaunchKernelGGL(k_bin_scatter, dim3(nblocks(n)), dim3(kBlock), 0, s, n, b);
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
                              unsigned long long *npairs, hipStream_t s) {
    hipLaunchKernelGGL(k_forces_rows, dim3(nblocks(n)), dim3(kBlock), 0, s, n, cnt, cap_c, dist, tan, cutoff, kind, k,
                       sigma, F, Ei, npairs);
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
    hipLaunchKernelGGL(k_integrate, dim3(nblocks(n)), dim3(kBlock), 0, s, n, m.V, m.T, m.fnrm, face, F, kind, dt,
                       mobility, kT, friction, seed, step, disp);
    return hipGetLastError();
}

}  // namespace gsim
