/*
 * CPU FP64 oracle for the geodesic-interaction hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may include, link,
 * load or call this code: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do. It shares no code with the HIP library.
 *
 * What it computes, and the passages it follows (arXiv 2404.19751):
 *  - mesh half-edge structure, corner-angle sums, pseudo-source vertices
 *    (Sec. 2.2: triangulated surface; Sec. 3.2: spherical vertices have angle
 *    sum < 2 pi);
 *  - exact polyhedral geodesic distance and initial unit tangent for every
 *    particle pair closer than a cutoff (Sec. 2.2, the MMP idea of
 *    considering all local unfoldings; Sec. 3.1, distances l_ij and tangents
 *    at the source; submeshing by the Euclidean lower bound). This is the plain
 *    definition written out: a shortest path is a chain of straight segments
 *    in planar unfoldings, bending only at saddle or boundary vertices; every
 *    such chain shorter than the cutoff is enumerated by brute force, with no
 *    trimming, and the shortest kept (Dijkstra over the bend vertices);
 *  - the same distances by the window-propagation method itself (Sec. 2.2:
 *    MMP's continuous Dijkstra with windows trimmed to the pointwise
 *    minimum), with its counts of windows;
 *  - the per-particle straight walk across faces with parallel transport of
 *    the velocity (Sec. 3.2, the shift algorithm and its steps (a)-(d));
 *  - Philox4x32-10 (Salmon et al., SC'11) for Brownian noise (Sec. 2.1);
 *  - the in-surface (restricted Euclidean) Voronoi neighbours of the
 *    particles, from which Sec. 5 counts coordination numbers and defects:
 *    per triangle, the bisector segment of every candidate pair clipped by
 *    the half-spaces of every other particle.
 */
#ifndef GSIM_ORACLE_H
#define GSIM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_mesh orc_mesh;
typedef struct orc_pairs orc_pairs;

/* 0 = ok; 1 = bad argument; 2 = non-manifold edge; 3 = inconsistent
 * orientation; 4 = non-manifold vertex; 5 = degenerate face. */
int orc_mesh_build(int nv, const double *V, int nf, const int *T, orc_mesh **out);
void orc_mesh_free(orc_mesh *m);
/* twin[3nf], theta[nv] (corner-angle sum), pseudo[nv], boundary[nv] */
void orc_mesh_export(const orc_mesh *m, int *twin, double *theta, unsigned char *pseudo, unsigned char *boundary);

/* Geodesic neighbour pairs (i -> j, j != i, d_ij < cutoff) for the sources
 * listed in `src` (all particles if src == NULL). cutoff <= 0 or infinite
 * means "all pairs" (only sensible on small meshes). nthreads <= 0: OpenMP
 * default. tie_rel: every initial direction of a path within tie_rel * d of
 * the shortest is kept in the pair's tie set (<= 0: 1e-9); a pair whose set
 * has more than one direction is flagged as a tie. cone_slack: a target
 * counts as inside a straight link's cone when its direction is within the
 * angle whose sine is cone_slack (<= 1e-12: 1e-12), so the tie set also
 * holds the directions of straight links to points that close to the
 * target (the resolution of a reduced-precision computation). Returns NULL
 * on bad input. */
orc_pairs *orc_geodesic_pairs(const orc_mesh *m, int n, const int *face, const double *bary, double cutoff,
                              int nsrc, const int *src, int nthreads, double tie_rel, double cone_slack);
int64_t orc_pairs_count(const orc_pairs *p);
int64_t orc_pairs_tie_count(const orc_pairs *p);
/* off[nsrc+1], nbr[P], dist[P], tan[P][3], flags[P], tie_off[P+1], tie_tan[T][3]
 * and tie_dist[T] (the length of the shortest path found in each direction) */
void orc_pairs_export(const orc_pairs *p, int64_t *off, int32_t *nbr, double *dist, double *tan, uint8_t *flags,
                      int64_t *tie_off, double *tie_tan, double *tie_dist);
/* counters: [0] windows processed, [1] windows pruned by the bound,
 * [2] roots expanded, [3] pseudo-source distance improvements, [4] sources
 * rejected (position on a vertex) */
void orc_pairs_counters(const orc_pairs *p, int64_t *c5);
void orc_pairs_free(orc_pairs *p);

/* The same pairs by the exact window-propagation method of Sec. 2.2 (the
 * continuous Dijkstra of Mitchell, Mount & Papadimitriou with windows
 * trimmed to the pointwise minimum on every edge, pseudo-source vertices
 * launched once): an independent route to the distances of
 * orc_geodesic_pairs and the method's own count of work. One direction per
 * pair (the first shortest found; no tie sets: tie_off[p] = p). Returns NULL
 * on bad input. */
orc_pairs *orc_geodesic_pairs_windows(const orc_mesh *m, int n, const int *face, const double *bary, double cutoff,
                                      int nsrc, const int *src, int nthreads);
/* counters of orc_geodesic_pairs_windows, summed over sources: [0] windows
 * inserted, [1] windows propagated, [2] windows trimmed (shortened, split or
 * removed), [3] pseudo-source launches, [4] faces entered (per source),
 * [5] insertions dropped (dominated or beyond the bound), [6] sources
 * rejected (on a vertex) */
void orc_pairs_window_counters(const orc_pairs *p, int64_t *c7);

/* Per-particle walk (shift). disp[n][3] (normal part removed inside), vel may
 * be NULL. face/bary/vel updated in place. stats[5]: crossings, vertex hits,
 * boundary hits, iteration-cap hits, near-vertex passes. flags[n] (may be
 * NULL): bit0 vertex hit, bit1 near-vertex pass, bit2 cap hit, bit3 boundary. */
int orc_walk(const orc_mesh *m, int n, int *face, double *bary, const double *disp, double *vel, int64_t *stats,
             uint8_t *flags);

/* Restricted Voronoi neighbours (Sec. 5): adj[n][n] = 1 where the surface
 * points equidistant (3D) from particles i and j and no farther from them
 * than from any other particle form a set longer than tol. xyz[n][3] are
 * points on the mesh. 0 = ok, 1 = bad argument. */
int orc_voronoi_pairs(const orc_mesh *m, int n, const double *xyz, double tol, unsigned char *adj);

/* Philox4x32-10: out[4] for counter ctr[4] and key key[2]. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

#ifdef __cplusplus
}
#endif
#endif
