// Internal declarations shared by the host API and the kernel translation
// units of the gsim library. Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace gsim {

// Per-half-edge unfolding record. Half-edge h = 3f + k runs from vertex
// T[f][k] (A) to T[f][(k+1)%3] (B); face f lies on its left. The "edge frame"
// of h has its origin at A, x along A->B, y towards the opposite vertex C.
struct alignas(16) HeRec {
    double L;    // |AB|
    double cx;   // C in the edge frame (cy > 0)
    double cy;
    double Lp;   // |CA| = length of prev(h)
    double Ln;   // |BC| = length of next(h)
    double ex, ey;  // (cx, cy) / Lp: axis of the frame on edge A->C, seen from h's frame
    double ux, uy;  // (L - cx, -cy) / Ln: axis of the frame on edge C->B
    int32_t tn;  // twin(next(h)) : the half-edge entered across BC, -1 on the boundary
    int32_t tp;  // twin(prev(h)) : the half-edge entered across CA
    int32_t opp_flags;  // (C << 1) | (C is a pseudo-source vertex)
    int32_t twin;       // twin(h)
    int32_t tail, head; // vertices A and B
};
static_assert(sizeof(HeRec) == 96, "HeRec must be a 96-byte record");

// FP32 copy of the geometric part (FP32-mixed mode).
struct alignas(16) HeRecF {
    float L, cx, cy, Lp;
    float Ln, ex, ey, ux;
    float uy;
    int32_t tn, tp;
    int32_t opp_flags;  // (opp << 1) | pseudo
};
static_assert(sizeof(HeRecF) == 48, "HeRecF must be 48 bytes");

enum : uint8_t { VF_PSEUDO = 1, VF_BOUNDARY = 2 };
enum : uint8_t { GSIM_PAIR_TIE_BIT = 1, GSIM_PAIR_ZERO_BIT = 2, GSIM_PAIR_GUARD_BIT = 4 };
// Per-particle flags of the last walk, step or force call (the same bits as
// the public GSIM_PF_* values).
enum : uint8_t { PF_VERTEX = 1, PF_NEAR_VERTEX = 2, PF_CAP = 4, PF_BOUNDARY = 8, PF_NONFINITE = 16 };

// Per bend vertex (dense number): its position and its fan of outgoing
// half-edges, read together when the vertex is launched.
struct PseudoRec {
    double x, y, z;
    int32_t v, fan_beg, fan_deg, pad;
};
static_assert(sizeof(PseudoRec) == 40, "PseudoRec must be a 40-byte record");

struct DevMesh {
    int32_t nv = 0, nf = 0;
    double *V = nullptr;        // [nv][3]
    int32_t *T = nullptr;       // [nf][3]
    HeRec *he = nullptr;        // [3nf]
    int32_t *twin = nullptr;    // [3nf] twin of each half-edge (-1 on the boundary), 12 bytes a face
    HeRecF *hef = nullptr;      // [3nf]
    uint8_t *vflag = nullptr;   // [nv]
    double *theta = nullptr;    // [nv] corner-angle sum
    int32_t *fan_off = nullptr; // [nv+1]
    int32_t *fan = nullptr;     // [3nf] outgoing half-edges, CCW, boundary fans start clockwise-most
    double *corner = nullptr;   // [3nf] corner angle of face h/3 at the tail of h
    double *fnrm = nullptr;     // [nf][3] unit outward normal
    double *fpos = nullptr;     // [nf][18]: the face's vertex positions in slot order, then the unit
                                // directions of its half-edges 3f+0..2
    int32_t *pidx = nullptr;    // [nv] bend-vertex number (0..n_pseudo-1) of a pseudo-source, else -1
    int32_t *pvert = nullptr;   // [max(n_pseudo,1)] the vertex of each bend-vertex number
    PseudoRec *prec = nullptr;  // [max(n_pseudo,1)] its position and fan
    double bbmin[3], bbmax[3];
    double mean_edge = 0, min_edge = 0, max_edge = 0;
    int32_t n_boundary_edges = 0, n_pseudo = 0;
};

// Host-side mesh analysis (mesh_build.cpp).
struct HostMesh {
    int nv = 0, nf = 0;
    std::vector<double> V;
    std::vector<int32_t> T;
    std::vector<int32_t> twin;
    std::vector<HeRec> he;
    std::vector<HeRecF> hef;
    std::vector<uint8_t> vflag;
    std::vector<double> theta, corner, fnrm, fpos;
    std::vector<int32_t> fan_off, fan;
    std::vector<int32_t> pidx, pvert;
    std::vector<PseudoRec> prec;
    double bbmin[3], bbmax[3];
    double mean_edge = 0, min_edge = 0, max_edge = 0;
    int32_t n_boundary_edges = 0, n_pseudo = 0;
};
// Returns empty string on success, else the reason the mesh is rejected.
std::string build_host_mesh(int nv, const double *xyz, int nf, const int32_t *tri, HostMesh &out);

// ---------------------------------------------------------------- kernels
struct PrefilterBufs {
    double *xyz;          // [n][3]
    int32_t *cell_of;     // [n]
    int32_t *cell_start;  // [ncell+1]
    int32_t *cell_fill;   // [ncell]
    int32_t *order;       // [n] particles sorted by cell
    int32_t *cand_cnt;    // [n] candidates per source (may exceed cap_c: overflow)
    int32_t *cand;        // [n][cap_c] candidate rows, sorted by j
    int cap_c;
    int32_t dims[3];
    double cell;
};

struct GeoParams {
    double cutoff;        // > 0, finite
    double launch_delta;  // bend-vertex launch bucket width
    double cone_tol;      // relative closed-cone slack
    double tie_rel;       // tie gap (relative)
    double tie_dir;       // two candidate tangents closer than this (rad) are the same direction
    double guard_rel;     // FP32 results this close (relative) to the cutoff are recomputed in FP64
    double cone_tol32, tie_rel32, tie_dir32;  // the FP32 pass's counterparts
    double bucket;        // all-pairs: key width of one processing round (0 = two max edge lengths)
    double dom_rel, dom_rel32;  // all-pairs: vertex-path domination margins (FP64 pass / FP32 pass)
    double slack32;       // FP32 pass: acceptance slack beyond the cutoff, relative to it
    double root_rel32;    // FP32 pass: a bend vertex is re-launched only when its distance improves by more
                          // than this fraction (FP32 rounding makes equal paths differ by ~1e-7)
    int32_t eager;        // launch bend vertices as soon as they are found
    int32_t stack_cap;    // windows per stack slot
    int32_t max_windows;  // per-source work limit
};

struct GeoOut {
    double *dist;   // [cand_cap]  (cand layout)
    double *tan;    // [cand_cap][3]
    uint8_t *flags; // [cand_cap]
};

struct alignas(128) Counters {  // device-side, int64; one 128-byte line
    unsigned long long windows, pruned, launches, stale, guards, nbr_pairs, limited, max_depth;
    unsigned long long nonfinite;  // particles that met a non-finite force, displacement or velocity
    unsigned long long crossings;  // edge crossings of the walks of time steps
};
static_assert(sizeof(Counters) == 128, "one counter slot per 128-byte line");
// The device counters are kCtrSlots copies, one line each: each workgroup
// of the geodesic grid adds into copy (workgroup mod kCtrSlots), so that its
// end-of-workgroup atomics do not serialise on one line; the other kernels
// add into the first; the host sums them (max_depth: the maximum).
constexpr int kCtrSlots = 64;
constexpr int kCtrStride = 1;  // Counters between two slots
constexpr int kCtrWords = (int)(sizeof(Counters) / 8);  // 64-bit words of one slot

// launchers (return hipError_t of the launch)
hipError_t launch_xyz(const DevMesh &m, int n, const int32_t *face, const double *bary, double *xyz,
                      hipStream_t s);
hipError_t launch_zero_i32(int32_t *p, int64_t n, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s);
hipError_t launch_scan_i32_to_i64(const int32_t *in, int64_t *out, int n, int64_t *scratch, hipStream_t s);

// One surface of a batch (a single surface is a batch of one): everything
// the binning, geodesic and update kernels read or write for it. The host
// fills it; kernels read it from a device-resident table.
struct SurfDesc {
    DevMesh m;
    int32_t n;          // particles on the surface
    int32_t src_begin;  // index of its first source in the batch
    int32_t *face;
    double *bary, *vel, *xyz;
    // next state, written by the cutoff kernel's fused update (time steps
    // with a cutoff and a non-FIRE integrator) while other sources still
    // read the current one; a commit kernel copies it back after the pass
    int32_t *face_out;
    double *bary_out, *vel_out;
    // prefilter cell grid (cells no smaller than the cutoff)
    int32_t *cell_of, *cell_start, *order;
    int32_t dims[3];
    double cell, lo[3];
    // candidate rows [n][cap], sorted by j (all-pairs: row i holds every j)
    int32_t cap;
    int32_t all_pairs;  // no cutoff: every other particle is a target
    int32_t *cand_cnt, *cand;
    double *cdist, *ctan;
    uint8_t *cflags;
    double cutoff, cut2;
    // particles by face (all-pairs target lookup): forder[fstart[f] .. fstart[f+1])
    int32_t *fstart, *forder;
    // potential and integrator of the fused update
    int32_t pkind, ikind;
    double pk, psigma, dt, mobility, kT, friction;
    uint64_t seed;
    // FIRE: parameters, forces of the current iteration, state on the device
    double max_disp, dt_max, alpha0, f_alpha, f_inc, f_dec;
    int32_t n_min;
    double *F;                // [n][3]
    struct FireState *fire;
    uint64_t *step;  // device counter: index of the current step since the particles were set
                     // (all ones before the first; each step's pass moves it on first)
    uint8_t *wflags;
    long long *prof;  // optional per-source profile [n][8]
};

// Capacity of a candidate row: the most Euclidean candidates one source may
// have with its targets in an LDS table of the geodesic kernel. Batches with
// more use the kernel's big-candidate instantiation (targets in global
// memory, rows as wide as the largest count needs), up to kBigCandMax.
constexpr int kCandCap = 128;
constexpr int kBigCandMax = 4096;
// Most particles on one surface in whole-mesh passes. The rows hold n x n
// pair slots of 37 bytes (indices are 64-bit): about 79 GB at this count,
// and a pairs call's compacted output up to as much again, which fits one
// 288 GB device. Each pass also checks the memory actually free first.
constexpr int kAllPairsMax = 46340;

// FIRE state of one surface (device memory): time step, mixing factor,
// consecutive iterations with positive power, and the mixing coefficients
// of the current iteration (v <- cv v + cf F).
struct FireState {
    double dt, alpha, cv, cf;
    int32_t n_pos, init;
};

constexpr int kMaxBatch = 64;
// Surface boundaries of a batch, passed by value: surface s owns the
// flattened indices [begin[s], begin[s+1]).
struct BatchIdx {
    int32_t nsurf;
    int32_t begin[kMaxBatch + 1];
};
__device__ inline int batch_surface(const BatchIdx &b, int idx) {
    int lo = 0, hi = b.nsurf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.begin[mid] <= idx) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Geodesic launch shape (chosen by hand or by the autotuner; results do not
// depend on it).
struct GeoShape {
    int32_t lds_stack_kb;  // LDS window stack per wavefront: 4, 8 or 16 KiB
    int32_t nslots;        // resident wavefronts of the persistent grid
    int32_t grab;          // consecutive sources a wavefront claims at a time
    int32_t pad_lds;       // extra LDS bytes per workgroup (spreads a small grid over every compute unit)
};

// Candidate search (Euclidean prefilter) and geodesics for every source of
// the batch, one wavefront per source. The cell lists must be current.
// With `fuse`, each source particle is also moved (force from its row,
// integrator, walk) into the next-state arrays once its row is final. Non-null
// ev0/ev1 are recorded by the dispatch at the kernel's start and end.
// gcap > 0 selects the big-candidate instantiation: every surface's rows are
// sd.cap wide (at most kBigCandMax) and each resident wavefront keeps its
// source's target arrays for up to gcap targets in gtab
// (geodesic_gtab_bytes(gcap) bytes per wavefront). group = 2, 4 or 8: with
// more sources than slots, that many sources per wavefront (the bend-vertex
// tables then hold rcap = group times the bend vertices of a surface).
hipError_t launch_geodesic(const SurfDesc *desc, const BatchIdx &bi, const GeoParams &gp, const GeoShape &shape,
                           char *stack_mem, char *roots, int64_t rstride, int rcap, int32_t *work_ctr, Counters *ctr,
                           bool fp32, bool fuse, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                           char *gtab = nullptr, int gcap = 0, int group = 1, bool pre_cand = false);
// The Euclidean candidate rows and counts of every source of the batch,
// group sources at a time (2, 4 or 8), ahead of a grouped geodesic pass
// (launched with pre_cand), which then reads them instead of searching.
hipError_t launch_candidates(const SurfDesc *desc, const BatchIdx &bi, int group, hipStream_t s);
int64_t geodesic_gtab_bytes(int gcap);
// All-pairs geodesics (no cutoff) for every source of the batch: every other
// particle of the surface is a target. vdist: per resident wavefront a table
// of vstride vertex distances; roots: per resident wavefront a bend-vertex
// table of rstride bytes for rcap bend vertices (bend_table_bytes); ttab:
// per resident wavefront the state of tcap targets (4 doubles each).
hipError_t launch_geodesic_all(const SurfDesc *desc, const BatchIdx &bi, const GeoParams &gp, const GeoShape &shape,
                               char *stack_mem, double *vdist, int64_t vstride, char *roots, int64_t rstride,
                               int rcap, double2 *ttab, int tcap, int32_t *work_ctr, Counters *ctr, bool fp32,
                               hipStream_t s);
// In-surface Voronoi neighbours (k_voronoi.hip): at most kVoronoiMax
// particles (an n x n adjacency bitset). launch_voronoi_faces marks every
// pair of particles whose cells share a boundary longer than tol; cell lists
// of a grid with origin lo (cell size `cell`, dims) over xyz; err[0] counts
// faces with too many candidates, err[1] cells with too many vertices.
constexpr int kVoronoiMax = 32768;
hipError_t launch_voronoi_faces(const DevMesh &m, int n, const double *xyz, const int32_t *cell_start,
                                const int32_t *order, const int dims[3], const double lo[3], double cell,
                                unsigned long long *bits, int64_t words, double tol, int32_t *err, hipStream_t s);
hipError_t launch_voronoi_count(const unsigned long long *bits, int n, int64_t words, int32_t *cnt, hipStream_t s);
hipError_t launch_voronoi_fill(const unsigned long long *bits, int n, int64_t words, const int64_t *off, int32_t *nbr,
                               hipStream_t s);
// Bytes of one wavefront's bend-vertex table for rcap bend vertices (both
// geodesic kernels): five doubles and four int32 each, rounded up to 256
// bytes.
// bytes of one wavefront's bend-vertex table: rcap records of kBendRec bytes
// and three int32 lists of rcap entries
constexpr int kBendRec = 48;
__host__ __device__ inline int64_t bend_table_bytes(int rcap) {
    return ((int64_t)rcap * (kBendRec + 12) + 255) / 256 * 256;
}
// Set nslots bend-vertex tables (rstride bytes, rcap vertices each) to
// empty: every distance infinite, nothing queued. The kernels leave them
// empty again after each source.
hipError_t launch_bend_init(char *roots, int nslots, int64_t rstride, int rcap, hipStream_t s);
int geodesic_all_blocks_per_cu(int lds_stack_kb, bool fp32);
// particles of one surface sorted by face (counting sort; counts must be zeroed)
hipError_t launch_face_sort(const SurfDesc &d, int32_t *counts, int64_t *tmp64, int64_t *scan_scratch, hipStream_t s);
// row i of an all-pairs surface lists every particle j in order
hipError_t launch_identity_rows(int n, int cap, int32_t *cand_cnt, int32_t *cand, hipStream_t s);
// FIRE: forces and the power / norm reduction of every FIRE surface (blk:
// blocks of 256 particles per surface), then the control step
constexpr int kFireBlock = 256;
hipError_t launch_fire_control(const SurfDesc *desc, const BatchIdx &blk, double *partials, Counters *ctr,
                               hipStream_t s);

// LDS bytes of one geodesic workgroup for a stack size (occupancy planning)
size_t geodesic_lds_bytes(int lds_stack_kb, bool fp32, bool big = false);
// positions + cell counting sort, one workgroup per surface (every surface's
// grid must have at most kSmallCells cells)
constexpr int kSmallCells = 4096;
// Work counters of the persistent geodesic grids: one per XCD chunk, each on
// a 128-byte line of its own so that claims on different chunks do not
// contend.
constexpr int kWorkChunks = 8;
constexpr int kWorkStride = 32;  // int32 entries between two chunks' counters
constexpr int kWorkInts = kWorkChunks * kWorkStride;
// (also clears the work counters and, when `advance`, moves every surface's
// step counter on by one)
// commit: take the state from the next-state arrays first (fused time steps)
hipError_t launch_bin_batch(const SurfDesc *desc, int nsurf, int32_t *work, bool advance, bool commit,
                            hipStream_t s);
// the same start of a pass without the binning
hipError_t launch_pass_begin(const SurfDesc *desc, int nsurf, int32_t *work, bool advance, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s);
// fused force + integrator + walk for every particle of the batch
hipError_t launch_update_batch(const SurfDesc *desc, const BatchIdx &bi, int block, Counters *ctr,
                               hipStream_t s);
// next state -> current state for every particle of the batch
hipError_t launch_commit_batch(const SurfDesc *desc, const BatchIdx &bi, hipStream_t s);
// Counting sort of n particles into the cells of b: positions, each
// particle's cell, the cells' starts (cell_start[ncell] = n) and the
// particles in cell order. b.cell_fill must hold zeros (clear writes them
// first) and holds zeros again afterwards. With work, the first workgroup
// also starts a geodesic pass of the one surface desc[0] (its work
// counters; with advance, its step counter).
hipError_t launch_cell_sort(const DevMesh &m, int n, const int32_t *face, const double *bary, PrefilterBufs &b,
                            int64_t *scratch, bool clear, const SurfDesc *desc, int32_t *work, bool advance,
                            hipStream_t s);
// resident geodesic workgroups per compute unit for a stack size (0 on error)
int geodesic_blocks_per_cu(int lds_stack_kb, bool fp32, bool big = false);

hipError_t launch_i64_to_i32(const int64_t *in, int32_t *out, int n, hipStream_t s);

hipError_t launch_count_rows(int n, const int32_t *cnt, int cap_c, const double *dist, double cutoff, int32_t *out,
                             hipStream_t s);
hipError_t launch_compact_rows(int n, const int32_t *cnt, int cap_c, const int32_t *cand, const double *dist,
                               const double *tan, const uint8_t *flags, double cutoff, const int64_t *off,
                               int32_t *nbr, double *odist, double *otan, uint8_t *oflags, hipStream_t s);
// F_i and E_i from the rows; pflags[i] (may be null) receives PF_NONFINITE
// when either is not finite, and nonfinite counts such particles.
hipError_t launch_forces_rows(int n, const int32_t *cnt, int cap_c, const double *dist, const double *tan,
                              double cutoff, int kind, double k, double sigma, double *F, double *Ei,
                              unsigned long long *npairs, uint8_t *pflags, unsigned long long *nonfinite,
                              hipStream_t s);
// Checks a particle state before it is used: bad[0] counts face indices
// outside [0, nf), bad[1] barycentric triples that are not finite, outside
// [0, 1], do not sum to 1 within 1e-9 or put the particle on a vertex,
// bad[2] velocities (vel may be null) that are not finite. bad[0..2] must be
// zero beforehand.
hipError_t launch_validate_state(int nf, int n, const int32_t *face, const double *bary, const double *vel,
                                 int32_t *bad, hipStream_t s);
// cnt[i] = the particles j != i within sqrt(cut2) of particle i, from the
// cell lists in b (cells no smaller than the cutoff)
hipError_t launch_count_candidates(int n, const PrefilterBufs &b, double cut2, int32_t *cnt, hipStream_t s);
hipError_t launch_sum(const double *x, int n, double *out, double *scratch, hipStream_t s);
hipError_t launch_integrate(const DevMesh &m, int n, const int32_t *face, const double *F, int kind, double dt,
                            double mobility, double kT, double friction, uint64_t seed, uint64_t step,
                            double *disp, hipStream_t s);
// The walk of every particle; stats[8] (zeroed beforehand) receive the
// crossings, vertex hits, boundary hits, crossing-cap hits, near-vertex
// passes and the particles left in place because their displacement or
// velocity was not finite; flags[n] (may be null) the PF_* bits.
hipError_t launch_walk(const DevMesh &m, int n, int32_t *face, double *bary, const double *disp, double *vel,
                       unsigned long long *stats, uint8_t *flags, hipStream_t s);
// The same walk with its statistics reduced without atomics: one row of 8
// counts per workgroup of kWalkBlock particles in part[ceil(n / kWalkBlock)][8],
// then their column sums, in a fixed order, in tot[8]. Nothing needs
// clearing beforehand; flags may be null.
constexpr int kWalkBlock = 256;
hipError_t launch_walk_blocks(const DevMesh &m, int n, int32_t *face, double *bary, const double *disp, double *vel,
                              uint8_t *flags, unsigned long long *part, unsigned long long *tot, hipStream_t s);

}  // namespace gsim
