/*
 * gsim: geodesic-interaction hot path for particles on triangulated
 * surfaces, for AMD MI355X (gfx950).
 *
 * Reference method: Webb & Sussman, "curvedSpaceSim: A framework for
 * simulating particles interacting along geodesics" (arXiv 2404.19751).
 * The operations exported here are the paper's two primitives for mesh
 * spaces: "displacement" (geodesic distances l_ij and the tangent directions
 * at the source, Sec. 2.1 last paragraph and Sec. 3.1) and "shift" (moving a
 * particle straight across faces, rotating the displacement and the velocity
 * about every crossed edge, Sec. 3.2), plus the force sum of Sec. 3.1 and the
 * overdamped / Brownian updates of Sec. 2.1.
 *
 * Conventions shared by every call
 *  - A particle position is a face index plus a barycentric triple of
 *    doubles (Sec. 3, mesh-space models), bary[k] weighting the face's k-th
 *    vertex tri[f][k]. Triples must be >= 0 and sum to 1 (to rounding).
 *  - Vectors (forces, displacements, velocities, tangents) are 3D and lie in
 *    the plane of the particle's current face (Sec. 3.2, first paragraph).
 *  - Faces are listed counter-clockwise seen from outside (outward normals).
 *  - Host pointers are borrowed for the duration of the call only and never
 *    retained; device state is owned by the context. Calls named *_dev take
 *    device pointers (e.g. a torch tensor's data_ptr) and are ordered on the
 *    context's stream.
 *  - Every call returns a gsim_status; nothing throws or aborts across the
 *    ABI. gsim_last_error() describes the last failure on a context.
 *  - A context is not thread-safe; its precision is fixed at creation.
 *  - Every call makes the context's device current for its duration and then
 *    restores the caller's current device.
 */
#ifndef GSIM_H
#define GSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsim_ctx gsim_ctx;

typedef enum {
    GSIM_OK = 0,
    GSIM_E_ARG = -1,      /* bad argument (null pointer, size, unknown id, out-of-range face) */
    GSIM_E_MESH = -2,     /* mesh not a 2-manifold, inconsistently oriented, or a face angle < 1e-6 rad */
    GSIM_E_OOM = -3,      /* device allocation failed */
    GSIM_E_CAPACITY = -4, /* caller buffer too small: the required count is reported */
    GSIM_E_DEVICE = -5,   /* HIP runtime error */
    GSIM_E_STATE = -6,    /* e.g. no particles set on the mesh */
    GSIM_E_LIMIT = -7,    /* a per-source work limit was exceeded (see gsim_last_error) */
    GSIM_E_NONFINITE = -8 /* some particles met a non-finite (NaN or infinite) force, displacement or
                             velocity: they were left where they were, the call's other results stand,
                             and gsim_particle_flags marks them with GSIM_PF_NONFINITE */
} gsim_status;

typedef enum { GSIM_FP64 = 0, GSIM_FP32_MIXED = 1 } gsim_precision;

typedef struct {
    int32_t nv, nf;
    int32_t n_boundary_edges;
    int32_t n_pseudo_sources; /* saddle (angle sum >= 2 pi - 1e-9) or boundary vertices */
    double mean_edge, min_edge, max_edge;
    double bbox_min[3], bbox_max[3];
} gsim_mesh_info;

/* Neighbour pairs (i -> j, j != i, d_ij < cutoff) as CSR rows sorted by j.
 * The caller owns every buffer. On input `capacity` is the number of pair
 * entries nbr/dist/tan/flags can hold; on return `count` is the number of
 * pairs (also on GSIM_E_CAPACITY, so a second call can size the buffers). */
typedef struct {
    int64_t capacity;
    int64_t count;
    int64_t *off;   /* [n+1] */
    int32_t *nbr;   /* [capacity] neighbour index j */
    double *dist;   /* [capacity] geodesic distance d_ij */
    double *tan;    /* [capacity][3] unit tangent at i towards j, in the plane of i's face */
    uint8_t *flags; /* [capacity] GSIM_PAIR_* bits */
} gsim_pairs;

enum {
    GSIM_PAIR_TIE = 1,     /* a second, different initial direction is within the tie gap (cut locus) */
    GSIM_PAIR_ZERO = 2,    /* d == 0: tangent undefined, contributes no force */
    GSIM_PAIR_GUARD = 4    /* distance re-checked in FP64 near the cutoff (FP32-mixed mode) */
};

typedef enum { GSIM_POT_HARMONIC = 0, GSIM_POT_COULOMB = 1, GSIM_POT_GAUSSIAN = 2 } gsim_potential_kind;

/* harmonic: U = (k/2)(1 - d/sigma)^2 for d < sigma;  coulomb: U = k/d;
 * gaussian: U = k exp(-d^2 / 2 sigma^2) (Sec. 2.1). cutoff <= 0 or
 * non-finite means all pairs. */
typedef struct {
    int32_t kind;
    double k, sigma, cutoff;
} gsim_potential;

typedef enum {
    GSIM_INT_OVERDAMPED = 0,
    GSIM_INT_BROWNIAN = 1,
    GSIM_INT_FIRE = 2,
    GSIM_INT_VERLET = 3
} gsim_integrator_kind;

/* overdamped: D = mobility dt F.
 * brownian:   friction D = dt F + sqrt(2 kT friction dt) (eta1 ex + eta2 ey),
 *             eta from Philox4x32-10 with counter (particle, step lo, step hi, 0)
 *             and key (seed lo, seed hi), Box-Muller on two 53-bit uniforms.
 * fire:       FIRE energy minimisation (Bitzek et al., Phys. Rev. Lett. 97,
 *             170201 (2006)), unit masses, one step = one iteration: with the
 *             power P = sum F.v, P > 0 mixes v <- (1 - alpha) v + alpha |v| F/|F|
 *             (norms over the surface's particles) and after more than n_min
 *             such iterations in a row sets dt <- min(f_inc dt, dt_max),
 *             alpha <- f_alpha alpha; P <= 0 sets v <- 0, dt <- f_dec dt,
 *             alpha <- alpha0. Then v += dt F and each particle walks dt v
 *             (at most max_disp long), its velocity parallel-transported.
 *             dt is the initial step; the state restarts when particles are
 *             set. Zero fields select the defaults in brackets.
 * verlet:     velocity Verlet (Newton's equation, Sec. 2.1 Eq. (1); the NVE
 *             runs of Sec. 4) in leapfrog form with unit masses: the stored
 *             velocity is the half-step velocity v_{k-1/2}; a step kicks
 *             v += dt F(x_k) and walks dt v, the velocity parallel-transported
 *             (Sec. 3.2). The integer-time velocity is v_{k-1/2} + (dt/2) F(x_k).
 *             The scheme is time-reversible: restarting from
 *             -(v_{k-1/2} + dt F(x_k)) retraces the trajectory. */
typedef struct {
    int32_t kind;
    double dt, mobility, kT, friction;
    uint64_t seed;
    double max_disp;                      /* fire: [no cap] */
    double dt_max;                        /* fire: [10 dt] */
    double alpha0, f_alpha, f_inc, f_dec; /* fire: [0.1, 0.99, 1.1, 0.5] */
    int32_t n_min;                        /* fire: [5] */
} gsim_integrator;

/* Statistics of one walk: edge crossings, passes through a vertex, boundary
 * reflections, walks stopped by the 10^4-crossing cap, passes within 1e-9
 * mean edge lengths of a vertex, and particles left in place because their
 * displacement or velocity was not finite. */
typedef struct {
    int64_t crossings, vertex_hits, boundary_hits, cap_hits, near_vertex, nonfinite;
} gsim_walk_stats;

/* Per-particle flags (gsim_particle_flags): what the last walk, step or
 * force call on the mesh met for each particle. */
enum {
    GSIM_PF_VERTEX = 1,      /* the walk passed through a vertex (straightest rule, or reversal on the boundary) */
    GSIM_PF_NEAR_VERTEX = 2, /* the walk passed within 1e-9 mean edge lengths of a vertex */
    GSIM_PF_CAP = 4,         /* the walk stopped at the 10^4-crossing cap */
    GSIM_PF_BOUNDARY = 8,    /* the walk was reflected at a boundary edge */
    GSIM_PF_NONFINITE = 16   /* a non-finite force, displacement or velocity: the particle stayed */
};

/* ---- context ------------------------------------------------------------ */
/* device: HIP device ordinal. hip_stream: a hipStream_t to run on, or NULL for
 * a stream the context creates (default priority). */
gsim_status gsim_create(int device, gsim_precision prec, void *hip_stream, gsim_ctx **out);
void gsim_destroy(gsim_ctx *ctx);
const char *gsim_last_error(const gsim_ctx *ctx); /* valid until the next call on ctx */
gsim_status gsim_synchronize(gsim_ctx *ctx);

/* ---- mesh ----------------------------------------------------------------
 * Builds the half-edge structure, corner-angle sums, pseudo-source flags and
 * per-half-edge unfolding constants on the host and copies them to device
 * memory once. xyz[nv][3], tri[nf][3]. Returns GSIM_E_MESH for non-manifold
 * or inconsistently oriented input or a face with an angle below 1e-6 rad. */
gsim_status gsim_mesh_upload(gsim_ctx *ctx, int32_t nv, const double *xyz, int32_t nf, const int32_t *tri,
                             int32_t *mesh_id);
gsim_status gsim_mesh_info_get(gsim_ctx *ctx, int32_t mesh_id, gsim_mesh_info *out);

/* ---- particle state -------------------------------------------------------
 * A position is a face and a barycentric triple (Sec. 3, mesh-space models).
 * face[n], bary[n][3], vel[n][3] (NULL = zero velocities). The state is
 * checked before it is taken: every face index in [0, nf), every triple in
 * [0, 1] summing to 1 within 1e-9 and not on a vertex (two zero
 * coordinates), every velocity finite; otherwise GSIM_E_ARG and the previous
 * state is kept. Setting the particles restarts the step counter, the FIRE
 * state and the per-particle flags. */
gsim_status gsim_particles_set(gsim_ctx *ctx, int32_t mesh_id, int32_t n, const int32_t *face, const double *bary,
                               const double *vel);
/* any output pointer may be NULL; xyz[n][3] receives the 3D positions */
gsim_status gsim_particles_get(gsim_ctx *ctx, int32_t mesh_id, int32_t *face, double *bary, double *vel,
                               double *xyz);
/* The same with device arrays (e.g. torch tensors' data_ptr), checked on the
 * device with the same rules before anything uses them (the call waits for
 * the check). */
gsim_status gsim_particles_set_dev(gsim_ctx *ctx, int32_t mesh_id, int32_t n, const int32_t *face_dev,
                                   const double *bary_dev, const double *vel_dev);
gsim_status gsim_particles_get_dev(gsim_ctx *ctx, int32_t mesh_id, int32_t *face_dev, double *bary_dev,
                                   double *vel_dev);
/* flags[n]: the GSIM_PF_* bits of each particle from the last walk, step or
 * force call on the mesh (zero after gsim_particles_set). */
gsim_status gsim_particle_flags(gsim_ctx *ctx, int32_t mesh_id, uint8_t *flags);
gsim_status gsim_particle_flags_dev(gsim_ctx *ctx, int32_t mesh_id, uint8_t *flags_dev);

/* ---- hot path -------------------------------------------------------------
 * geodesic_pairs: exact polyhedral geodesic distance and initial unit tangent
 * for every pair closer than `cutoff` (Sec. 3.1: sequence-tree distances and
 * tangents relative to the source; submeshing by the Euclidean lower bound).
 * Euclidean prefilter, window propagation and target query run on the GPU;
 * the CSR is then copied to the caller's host buffers. */
gsim_status gsim_geodesic_pairs(gsim_ctx *ctx, int32_t mesh_id, double cutoff, gsim_pairs *out);
/* The same, with every buffer of `out` (off, nbr, dist, tan, flags) in device
 * memory, written on the context's stream (the call waits only to learn the
 * pair count; the copies into `out` are ordered on the stream). */
gsim_status gsim_geodesic_pairs_dev(gsim_ctx *ctx, int32_t mesh_id, double cutoff, gsim_pairs *out);

/* voronoi_neighbours: the in-surface Voronoi neighbours of the particles
 * (Sec. 5: the restricted Euclidean Voronoi diagram on the surface, from
 * which coordination numbers and 5/7-fold defects are read). The cell of a
 * particle is the set of surface points no farther (3D distance) from it
 * than from any other particle; two particles are neighbours when their cells
 * share a boundary longer than 1e-10 mean edge lengths. Output CSR in host
 * buffers: off[n+1] (int64), nbr[count] (int32, ascending per row, both
 * directions present). count receives the number of entries; capacity is
 * nbr's length (GSIM_E_CAPACITY, with count filled in, when too small).
 * At most 32768 particles; GSIM_E_LIMIT when a face has more than 64
 * candidate particles or a cell piece more than 16 vertices. */
gsim_status gsim_voronoi_neighbours(gsim_ctx *ctx, int32_t mesh_id, int64_t *off, int32_t *nbr, int64_t capacity,
                                    int64_t *count);

/* compute_forces: F_i = sum_j U'(d_ij) t_ij (Sec. 3.1 force sum; with t_ij
 * pointing from i towards j a repulsive potential pushes i away from j) and
 * E = (1/2) sum_i sum_j U(d_ij). force[n][3] host buffer; energy may be NULL.
 * Recomputes the pairs for the potential's cutoff. A particle whose force or
 * energy is not finite is flagged (GSIM_PF_NONFINITE) and the call returns
 * GSIM_E_NONFINITE with every force written. */
gsim_status gsim_compute_forces(gsim_ctx *ctx, int32_t mesh_id, const gsim_potential *pot, double *force,
                                double *energy);
/* The same into device buffers force_dev[n][3] and energy_dev[1] (may be
 * NULL), copied on the context's stream. */
gsim_status gsim_compute_forces_dev(gsim_ctx *ctx, int32_t mesh_id, const gsim_potential *pot, double *force_dev,
                                    double *energy_dev);

/* displace_on_surface: the shift (Sec. 3.2). disp[n][3] host buffer; its
 * component normal to the particle's face is removed first. With
 * transport_velocity != 0 the stored velocities are parallel-transported
 * along the walk. stats may be NULL. A particle whose displacement (or
 * transported velocity) is not finite stays where it is, is flagged
 * (GSIM_PF_NONFINITE), and the call returns GSIM_E_NONFINITE after moving
 * the others. */
gsim_status gsim_displace_on_surface(gsim_ctx *ctx, int32_t mesh_id, const double *disp, int transport_velocity,
                                     gsim_walk_stats *stats);
/* The same with disp_dev[n][3] in device memory, read by the walk kernel in
 * place (no staging copy). */
gsim_status gsim_displace_on_surface_dev(gsim_ctx *ctx, int32_t mesh_id, const double *disp_dev,
                                         int transport_velocity, gsim_walk_stats *stats);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it): the walk of
 * gsim_displace_on_surface_dev without any allocation. It reads disp_dev and
 * moves the particles already set on the mesh; flags_dev[n] (device memory,
 * may be NULL) receives each particle's GSIM_PF_* bits. Its statistics go
 * through a scratch array of 512 KiB that each GPU holds for the whole
 * process (one row of counts per 256 particles, summed in a fixed order),
 * which limits a call to 2,097,152 particles (GSIM_E_LIMIT beyond). Calls on
 * one GPU share that array: calls that overlap in time on one GPU, from any
 * context or stream, race and must be ordered by the caller. The result
 * equals gsim_displace_on_surface_dev's bit for bit. */
gsim_status gsim_displace_on_surface_noalloc(gsim_ctx *ctx, int32_t mesh_id, const double *disp_dev,
                                             int transport_velocity, uint8_t *flags_dev, gsim_walk_stats *stats);

/* step: nsteps full time steps on device (prefilter, window propagation,
 * query, forces, integrator, walk); state stays in device memory. The noise
 * counter of step k is the number of steps taken on this mesh since its
 * particles were last set (so a run can be resumed bit-identically). A
 * particle that meets a non-finite force, displacement or velocity stays
 * where it is and is flagged; the call then returns GSIM_E_NONFINITE at its
 * end (the other particles' steps stand). */
gsim_status gsim_step(gsim_ctx *ctx, int32_t mesh_id, const gsim_potential *pot, const gsim_integrator *integ,
                      int32_t nsteps);

/* step_batched: nsteps full time steps of several independent surfaces at
 * once (the same per-surface work as gsim_step, Sec. 3.1 and 3.2). Every
 * step is one binning, one geodesic and one update (or commit) launch for the whole
 * batch: the persistent geodesic grid takes sources from all surfaces, so
 * small surfaces share the GPU instead of leaving it idle. mesh_ids[nmesh]
 * (1..64 distinct meshes, each with particles), pots[nmesh], integs[nmesh].
 * With a finite cutoff, no FIRE surface in the batch and at most four
 * particles per compute unit in all, the update is fused into the geodesic
 * launch ("fuse_update", default 1): each source's wavefront moves its
 * particle (force from its row, integrator, walk) into a next-state array as
 * soon as its row is final; the next step's binning, or a commit launch after
 * the last step, makes that the current state. The results are bit-identical
 * to the separate update launch.
 * When timing is off and nsteps >= 2, groups of "graph_steps" steps are
 * captured once into a HIP graph and replayed (the capture is cached until
 * the batch, a buffer or a knob changes). gsim_step is the batch of one. */
gsim_status gsim_step_batched(gsim_ctx *ctx, int32_t nmesh, const int32_t *mesh_ids, const gsim_potential *pots,
                              const gsim_integrator *integs, int32_t nsteps);

/* ---- tuning ----------------------------------------------------------------
 * Knobs of the geodesic kernel (set by the autotuner or by hand; results stay
 * exact, only the amount of work or the launch shape changes):
 *   "launch_delta"  bend-vertex launch bucket width (0 = half the mean edge)
 *   "stack_cap"     window-stack capacity per resident wavefront, cutoff passes
 *                   (64 .. 4M records of 64 bytes; default 16384)
 *   "max_slots"     resident wavefronts of the persistent grid (1 .. 65536)
 *   "max_windows"   per-source work limit (GSIM_E_LIMIT beyond it)
 *   "cone_tol"      closed-cone slack relative to the edge length
 *   "tie_rel"       relative gap under which a pair is flagged as a tie
 *   "tie_dir"       tangents closer than this angle (rad) count as one direction
 *   "guard_rel"     FP32-mixed: relative band around the cutoff recomputed in FP64
 *   "slack32"       FP32-mixed: windows are kept up to this fraction beyond the
 *                   cutoff (1e-6 .. 1e-2; the larger of it and guard_rel is used)
 *   "root_rel32"    FP32-mixed: a bend vertex is re-launched only when its distance
 *                   improves by more than this fraction (<= 1e-4; distances may then
 *                   exceed the exact value by this fraction)
 *   "lds_stack_kb"  window-stack depth in LDS per wavefront: 4, 8 or 16 KiB (sets
 *                   how many wavefronts fit on a compute unit)
 *   "grab"          consecutive sources a wavefront claims at a time (1 .. 64)
 *   "group_sources" 4 (default), 8, 2 or 1: passes with a cutoff and more
 *                   sources than resident wavefronts propagate up to this many
 *                   neighbouring sources together in one wavefront (each with
 *                   its share of the LDS target table; a source with more
 *                   candidates than its share runs alone). The group shrinks
 *                   until every resident wavefront gets a full one, the
 *                   expected candidates of a source (the mean plus three
 *                   standard deviations of a Poisson count) fit a share,
 *                   and the resident wavefronts' bend-vertex tables (one
 *                   60-byte entry per bend vertex and source) fit the table
 *                   budget (a third of the device's memory, at most 96 GB). Results equal those of single
 *                   sources to rounding (separately compiled multiply-adds).
 *                   In FP32-mixed mode a group propagates in FP32 and each
 *                   of its sources with a pair in the guard band runs again
 *                   alone in FP64
 *   "update_block"  workgroup size of the separate update kernel: 64 (default),
 *                   128 or 256
 *   "fuse_update"   1 (default): time steps with a cutoff and few enough particles
 *                   move each particle inside the geodesic launch; 0: always a
 *                   separate update launch per step
 *   "graph_steps"   steps captured per HIP graph in step calls (0 = no graphs)
 *   "time_geodesic_only"  1: while timing is on, record events around the
 *                   geodesic stage only (each event record costs the stream a few
 *                   microseconds)
 *   "whole_mesh"    1: finite-cutoff passes also run on the whole-mesh kernel
 *                   below (windows pruned at the cutoff; no limit on candidates or
 *                   bend vertices per source; at most 46,340 particles per
 *                   surface, whose n x n pair rows take 37 bytes each: 79 GB
 *                   at that count, checked against the free device memory
 *                   before each pass, as a pairs call's output is before it
 *                   is written; GSIM_E_LIMIT names the bytes). Without
 *                   it, the cutoff kernel takes up to 4096 Euclidean candidates
 *                   per source: up to 128 in an LDS table, more with the targets
 *                   in global memory and rows sized from a count of the
 *                   candidates at the start of each call (GSIM_E_LIMIT beyond
 *                   4096, or when moving particles outgrow that count within a
 *                   call by more than a quarter plus 32)
 *   Whole-mesh passes (no cutoff, or "whole_mesh" = 1):
 *   "stack_cap_all" window records per resident wavefront (1024 .. 4M)
 *   "max_windows_all" per-source work limit
 *   "bucket"        key width of one processing round (0 = 16 max edge lengths,
 *                   4 on a surface with saddle or boundary vertices)
 *   "dom_rel", "dom_rel32"  margins of the vertex-path domination tests */
gsim_status gsim_tune_set(gsim_ctx *ctx, const char *name, double value);

/* autotune: times the geodesic pass of the given batch (current particle
 * state, pots[nmesh] cutoffs) for LDS stack depths {4, 8, 16} KiB x sources
 * per claim {1, 2, 4}, and the fused update kernel for workgroup sizes
 * {64, 128, 256} on a scratch copy of the particle state (integs[nmesh]);
 * keeps the fastest of each (best of `reps` runs) in the context. Particle
 * state is left unchanged; results of later calls do not depend on the
 * choice. out (may be NULL) receives [lds_stack_kb, grab, update_block,
 * best geodesic-pass ms]. */
gsim_status gsim_autotune(gsim_ctx *ctx, int32_t nmesh, const int32_t *mesh_ids, const gsim_potential *pots,
                          const gsim_integrator *integs, int32_t reps, double *out);

/* ---- instrumentation ------------------------------------------------------
 * Per-kernel timing with HIP events recorded on the context's stream, only
 * while enabled. name: "prefilter", "geodesic", "fire", "update", "commit", "compact",
 * "forces", "walk", "voronoi". avg_ms is the mean duration of the stage. */
gsim_status gsim_timing_enable(gsim_ctx *ctx, int on);
gsim_status gsim_timing_get(gsim_ctx *ctx, const char *name, double *avg_ms, int64_t *launches);
/* Work counters. Of the last call: [0] windows processed,
 * [1] windows pruned, [2] bend-vertex (pseudo-source) launches,
 * [3] stale windows dropped, [4] sources recomputed in FP64 (FP32-mixed
 * guard band), [5] neighbour pairs,
 * [6] sources over a work limit, [10] deepest window stack of a source
 * (records, LDS and overflow together), [11] particles that met a non-finite
 * value, [12] edge crossings of the walks of time steps. Summed over the
 * calls since timing was last enabled: [7] neighbour pairs, [8] windows,
 * [9] passes. c[13]. */
gsim_status gsim_counters_get(gsim_ctx *ctx, int64_t *c);
/* Per-source profile of the geodesic kernel, accumulated over the calls
 * made while it is on: out[n][8] = GPU clock cycles, propagation-loop
 * iterations, windows, bend-vertex launches, and the cycles spent in set-up
 * (prefilter, tables, seeding), propagation, launches and result write-out. gsim_source_profile(ctx, 1,
 * NULL, 0) starts it; gsim_source_profile(ctx, 0, out, n) copies it out
 * (n = particles of the profiled mesh) and stops it. */
gsim_status gsim_source_profile(gsim_ctx *ctx, int on, int64_t *out, int32_t n);

#ifdef __cplusplus
}
#endif
#endif
