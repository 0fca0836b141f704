// Per-particle device operations shared by the force, integrator and fused
// update kernels: the pair potentials, the force sum over a neighbour row,
// Philox4x32-10 noise and the displacement of each integrator.
#pragma once
#include <cmath>

#include "gsim_internal.h"

namespace gsim {

// One atomic add per wavefront: the lanes' values are summed by shuffles
// first, so that a grid's counts do not serialise on one address. Every lane
// of the wavefront must call it (lane = threadIdx.x mod 64).
__device__ inline void wave_atomic_add(unsigned long long *p, unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(p, v);
}

// U(d) and dU/dd. 0 harmonic: U = (k/2)(1 - d/sigma)^2 for d < sigma;
// 1 coulomb: U = k/d; 2 gaussian: U = k exp(-d^2 / (2 sigma^2)) (Sec. 2.1).
__device__ inline void pair_potential(int kind, double d, double k, double sigma, double &U, double &dU) {
    if (kind == 0) {
        if (d < sigma) {
            const double x = 1.0 - d / sigma;
            U = 0.5 * k * x * x;
            dU = -(k / sigma) * x;
        } else {
            U = 0.0;
            dU = 0.0;
        }
    } else if (kind == 1) {
        U = k / d;
        dU = -k / (d * d);
    } else {
        U = k * exp(-d * d / (2.0 * sigma * sigma));
        dU = -(d / (sigma * sigma)) * U;
    }
}

// F_i = sum_j U'(d_ij) t_ij and E_i = (1/2) sum_j U(d_ij) over the pairs of
// row i closer than the cutoff, in ascending j; np = number of such pairs.
__device__ inline void row_force(int i, const int32_t *__restrict__ cnt, int cap, const double *__restrict__ dist,
                                 const double *__restrict__ tan, double cutoff, int kind, double k, double sigma,
                                 double F[3], double &E, int &np) {
    F[0] = F[1] = F[2] = 0.0;
    E = 0.0;
    np = 0;
    const int m = min(cnt[i], cap);
    auto add = [&](double d, double t0, double t1, double t2) {
        if (!(d < cutoff)) return;
        ++np;
        if (!(d > 0.0)) return;
        double U, dU;
        pair_potential(kind, d, k, sigma, U, dU);
        F[0] += dU * t0;
        F[1] += dU * t1;
        F[2] += dU * t2;
        E += 0.5 * U;
    };
    // eight entries' loads issued together (those past the row's end
    // masked), then summed in ascending order
    for (int s = 0; s < m; s += 8) {
        const int64_t p = (int64_t)i * cap + s;
        double d[8], t[8][3];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const bool in = s + q < m;
            d[q] = in ? dist[p + q] : INFINITY;
            t[q][0] = in ? tan[3 * (p + q)] : 0.0;
            t[q][1] = in ? tan[3 * (p + q) + 1] : 0.0;
            t[q][2] = in ? tan[3 * (p + q) + 2] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) add(d[q], t[q][0], t[q][1], t[q][2]);
    }
}

// Philox4x32-10 (Salmon et al., SC'11): ten multiply-xor rounds with a Weyl
// key schedule.
__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Two unit normals for (step, particle): counter (i, step lo, step hi, 0),
// key (seed lo, seed hi); two 53-bit uniforms and Box-Muller.
__device__ inline void gaussian_pair(uint64_t seed, uint64_t step, int i, double &e1, double &e2) {
    uint32_t c[4] = {uint32_t(i), uint32_t(step), uint32_t(step >> 32), 0u};
    philox10(c, uint32_t(seed), uint32_t(seed >> 32));
    const double u1 = (double(c[0] >> 5) * 67108864.0 + double(c[1] >> 6)) * (1.0 / 9007199254740992.0);
    const double u2 = (double(c[2] >> 5) * 67108864.0 + double(c[3] >> 6)) * (1.0 / 9007199254740992.0);
    const double r = sqrt(-2.0 * log(1.0 - u1));
    double sn, cs;
    sincos(2.0 * M_PI * u2, &sn, &cs);
    e1 = r * cs;
    e2 = r * sn;
}

// Displacement of one particle in face f for one step (Sec. 2.1):
// 0 overdamped D = mobility dt F;
// 1 Brownian  lam D = dt F + sqrt(2 kT lam dt) (eta1 ex + eta2 ey), with
//   (ex, ey) the face frame (ex along the face's first edge).
__device__ inline void displacement(const DevMesh &m, int f, int i, const double F[3], int kind, double dt,
                                    double mob, double kT, double lam, uint64_t seed, uint64_t step, double D[3]) {
    if (kind == 0) {
        const double s = mob * dt;
        D[0] = s * F[0];
        D[1] = s * F[1];
        D[2] = s * F[2];
        return;
    }
    double e1, e2;
    gaussian_pair(seed, step, i, e1, e2);
    // the unit direction of the first edge from the face record (one load
    // after the face index, not the vertex indices and then the vertices)
    const double *u0 = m.fpos + 18 * (int64_t)f + 9;
    const double ex[3] = {u0[0], u0[1], u0[2]};
    const double *nn = m.fnrm + 3 * (int64_t)f;
    const double ey[3] = {nn[1] * ex[2] - nn[2] * ex[1], nn[2] * ex[0] - nn[0] * ex[2], nn[0] * ex[1] - nn[1] * ex[0]};
    const double amp = sqrt(2.0 * kT * lam * dt) / lam, a = dt / lam;
    for (int d = 0; d < 3; ++d) D[d] = a * F[d] + amp * (e1 * ex[d] + e2 * ey[d]);
}

}  // namespace gsim
