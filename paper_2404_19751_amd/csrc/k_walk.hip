// Kernels of the shift (arXiv 2404.19751, Sec. 3.2) and of the fused
// per-particle update of a time step; the walk itself lives in walk.h.
#include <cmath>

#include "gsim_internal.h"
#include "particle_ops.h"
#include "walk.h"

namespace gsim {
namespace {

// every lane of the wavefront calls it (wavefront sums, one atomic each)
__device__ inline void flush_counts(const WalkCounts &wc, unsigned long long *stats) {
    if (!stats) return;
    wave_atomic_add(&stats[0], wc.cross_n);
    wave_atomic_add(&stats[1], wc.vhit);
    wave_atomic_add(&stats[2], wc.bhit);
    wave_atomic_add(&stats[3], wc.cap);
    wave_atomic_add(&stats[4], wc.near);
    wave_atomic_add(&stats[5], wc.nonfinite);
}

__global__ __launch_bounds__(128) void k_walk(DevMesh m, int n, int32_t *__restrict__ face, double *__restrict__ bary,
                                              const double *__restrict__ disp, double *__restrict__ vel,
                                              unsigned long long *__restrict__ stats, uint8_t *__restrict__ flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    WalkCounts wc = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        int f = face[i];
        double b[3] = {bary[3 * i], bary[3 * i + 1], bary[3 * i + 2]};
        const bool hv = vel != nullptr;
        d3 v = hv ? ld3(vel + 3 * (int64_t)i) : d3{0, 0, 0};
        uint8_t fl = 0;
        walk_one(m, f, b, ld3(disp + 3 * (int64_t)i), v, hv, wc, fl);
        face[i] = f;
        bary[3 * i] = b[0];
        bary[3 * i + 1] = b[1];
        bary[3 * i + 2] = b[2];
        if (hv) {
            vel[3 * i] = v.x;
            vel[3 * i + 1] = v.y;
            vel[3 * i + 2] = v.z;
        }
        if (flags) flags[i] = fl;
    }
    flush_counts(wc, stats);
}

// The walk of every particle with its statistics in per-workgroup partial
// rows instead of atomics: part[blockIdx][0..7] = crossings, vertex hits,
// boundary hits, cap hits, near-vertex passes, non-finite particles, 0, 0.
// Every row is written, so nothing needs clearing beforehand.
__global__ __launch_bounds__(kWalkBlock) void k_walk_blocks(DevMesh m, int n, int32_t *__restrict__ face,
                                                           double *__restrict__ bary, const double *__restrict__ disp,
                                                           double *__restrict__ vel, uint8_t *__restrict__ flags,
                                                           unsigned long long *__restrict__ part) {
    __shared__ unsigned long long sh[6][kWalkBlock / 64];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    WalkCounts wc = {0, 0, 0, 0, 0, 0};
    if (i < n) {
        int f = face[i];
        double b[3] = {bary[3 * i], bary[3 * i + 1], bary[3 * i + 2]};
        const bool hv = vel != nullptr;
        d3 v = hv ? ld3(vel + 3 * (int64_t)i) : d3{0, 0, 0};
        uint8_t fl = 0;
        walk_one(m, f, b, ld3(disp + 3 * (int64_t)i), v, hv, wc, fl);
        face[i] = f;
        bary[3 * i] = b[0];
        bary[3 * i + 1] = b[1];
        bary[3 * i + 2] = b[2];
        if (hv) {
            vel[3 * i] = v.x;
            vel[3 * i + 1] = v.y;
            vel[3 * i + 2] = v.z;
        }
        if (flags) flags[i] = fl;
    }
    unsigned long long c[6] = {wc.cross_n, wc.vhit, wc.bhit, wc.cap, wc.near, wc.nonfinite};
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        unsigned long long x = c[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if ((threadIdx.x & 63) == 0) sh[k][wv] = x;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        unsigned long long t = 0;
        if (threadIdx.x < 6)
            for (int w = 0; w < kWalkBlock / 64; ++w) t += sh[threadIdx.x][w];
        part[8 * (int64_t)blockIdx.x + threadIdx.x] = t;
    }
}

// tot[0..7] = the column sums of part[nb][8], in a fixed order.
__global__ __launch_bounds__(256) void k_walk_total(const unsigned long long *__restrict__ part, int nb,
                                                   unsigned long long *__restrict__ tot) {
    __shared__ unsigned long long sh[8][256];
    for (int k = 0; k < 8; ++k) {
        unsigned long long t = 0;
        for (int r = threadIdx.x; r < nb; r += 256) t += part[8 * (int64_t)r + k];
        sh[k][threadIdx.x] = t;
    }
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int k = 0; k < 8; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 8) tot[threadIdx.x] = sh[threadIdx.x][0];
}

// One full particle update of a time step, fused: the force from the
// particle's neighbour row (Sec. 3.1 force sum), the displacement of the
// integrator (Sec. 2.1), and the walk (Sec. 3.2). Rows hold only distances
// and tangents computed before any particle moves, so particles are
// independent here. Returns the particle's neighbour-pair count; wc receives
// the walk's counts.
__device__ inline int update_one(const SurfDesc *__restrict__ desc, const BatchIdx &bi, int g, WalkCounts &wc) {
    const int si = batch_surface(bi, g);
    const SurfDesc &sd = desc[si];
    const int i = g - bi.begin[si];
    if (sd.ikind != 2) {
        double F[3], E;
        int np = 0;
        row_force(i, sd.cand_cnt, sd.cap, sd.cdist, sd.ctan, sd.cutoff, sd.pkind, sd.pk, sd.psigma, F, E, np);
        move_particle(sd, i, F, sd.face, sd.bary, sd.vel, wc);
        return np;
    }
    // FIRE: forces and the control step come from the FIRE kernels; mix,
    // semi-implicit Euler, displacement dt v capped at max_disp
    const FireState st = *sd.fire;
    const d3 F = ld3(sd.F + 3 * (int64_t)i);
    d3 v = ld3(sd.vel + 3 * (int64_t)i);
    v = st.cv * v + st.cf * F;
    v = v + st.dt * F;
    d3 Dv = st.dt * v;
    const double L = sqrt(dot(Dv, Dv));
    if (L > sd.max_disp) Dv = (sd.max_disp / L) * Dv;
    const double D[3] = {Dv.x, Dv.y, Dv.z};
    walk_store(sd, i, sd.face[i], D, v, sd.face, sd.bary, sd.vel, wc);
    return 0;
}

// One thread per particle of the flattened batch.
__global__ __launch_bounds__(256) void k_update_batch(const SurfDesc *__restrict__ desc, BatchIdx bi,
                                                     Counters *__restrict__ ctr) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    WalkCounts wc = {0, 0, 0, 0, 0, 0};
    const int np = g < bi.begin[bi.nsurf] ? update_one(desc, bi, g, wc) : 0;
    // the counts: one atomic per wavefront, not one per particle
    wave_atomic_add(&ctr->nbr_pairs, (unsigned long long)np);
    wave_atomic_add(&ctr->nonfinite, wc.nonfinite);
    wave_atomic_add(&ctr->crossings, wc.cross_n);
}

// The state that the cutoff kernel's fused update wrote (the next-state
// arrays) becomes the current state: one thread per particle of the batch.
__global__ void k_commit_batch(const SurfDesc *__restrict__ desc, BatchIdx bi) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= bi.begin[bi.nsurf]) return;
    const int si = batch_surface(bi, g);
    const SurfDesc &sd = desc[si];
    const int i = g - bi.begin[si];
    sd.face[i] = sd.face_out[i];
    for (int q = 0; q < 3; ++q) {
        sd.bary[3 * i + q] = sd.bary_out[3 * i + q];
        sd.vel[3 * i + q] = sd.vel_out[3 * i + q];
    }
}

}  // namespace

hipError_t launch_commit_batch(const SurfDesc *desc, const BatchIdx &bi, hipStream_t s) {
    const int total = bi.begin[bi.nsurf];
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_commit_batch, dim3((total + 255) / 256), dim3(256), 0, s, desc, bi);
    return hipGetLastError();
}

hipError_t launch_update_batch(const SurfDesc *desc, const BatchIdx &bi, int block, Counters *ctr, hipStream_t s) {
    const int total = bi.begin[bi.nsurf];
    if (total <= 0) return hipSuccess;
    if (block != 64 && block != 128 && block != 256) block = 128;
    hipLaunchKernelGGL(k_update_batch, dim3((total + block - 1) / block), dim3(block), 0, s, desc, bi, ctr);
    return hipGetLastError();
}

hipError_t launch_walk_blocks(const DevMesh &m, int n, int32_t *face, double *bary, const double *disp, double *vel,
                              uint8_t *flags, unsigned long long *part, unsigned long long *tot, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nb = (n + kWalkBlock - 1) / kWalkBlock;
    hipLaunchKernelGGL(k_walk_blocks, dim3(nb), dim3(kWalkBlock), 0, s, m, n, face, bary, disp, vel, flags, part);
    hipLaunchKernelGGL(k_walk_total, dim3(1), dim3(256), 0, s, part, nb, tot);
    return hipGetLastError();
}

hipError_t launch_walk(const DevMesh &m, int n, int32_t *face, double *bary, const double *disp, double *vel,
                       unsigned long long *stats, uint8_t *flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_walk, dim3((n + 127) / 128), dim3(128), 0, s, m, n, face, bary, disp, vel, stats, flags);
    return hipGetLastError();
}

}  // namespace gsim
