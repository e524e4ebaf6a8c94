/*
 * fpts -- general field evaluation ("findpts") on high-order quad, hex and
 * surface meshes, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Mittal, Parik, Dutta, Fischer, Kolev, Lottes, "General Field
 * Evaluation in High-Order Meshes on GPUs", arXiv 2501.12349.  This library
 * implements the processor-local path: Setup (Section 3.1, surface variants
 * Section 4.1-4.3), Find (Section 3.2, 3.2.1, 4.4) and Interpolate (Section
 * 3.3).  The multi-rank global map of Section 3.1.4 is not part of it.
 *
 * Conventions shared by every entry point
 *  - Status: 0 on success, a negative FPTS_E* value on error.  Errors never
 *    abort the process.  Invalid point coordinates (NaN, Inf, far away) are
 *    data, not errors: such points come back NOT_FOUND.
 *  - Pointers named d_* are device memory owned by the caller.  Every call
 *    only enqueues work on `stream` (a hipStream_t, NULL = default stream)
 *    and returns; the caller keeps the buffers alive until the stream has
 *    drained.  Host pointers (h_*) are read before the call returns.
 *  - All floating point data is IEEE double unless stated otherwise.
 *  - A mesh handle is read-only after setup.  Calls on one mesh from several
 *    streams may overlap as long as each call has its own workspace.
 */
#ifndef FPTS_H
#define FPTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Point codes c* of the computational coordinates (Section 3.2). */
enum {
    FPTS_INTERIOR = 0,   /* r* inside the open reference box (and, for
                            surfaces, squared distance below eps_d) */
    FPTS_BORDER = 1,     /* in some element's boxes, not interior to any:
                            closest point of the best element */
    FPTS_NOT_FOUND = 2   /* outside the boxes of every element */
};

/* Status codes. */
enum {
    FPTS_OK = 0,
    FPTS_EINVAL = -1,    /* bad argument (dimension, order, null pointer,
                            size out of range, workspace too small) */
    FPTS_ENOMEM = -2,    /* host or device allocation failed */
    FPTS_EDEVICE = -3,   /* HIP error (launch failure, sticky error, no
                            device) */
    FPTS_EUNSUPPORTED = -4 /* valid request this build has no kernel for */
};

/* Newton precision of fpts_find. */
enum {
    FPTS_FP64 = 0,       /* every Newton pass in FP64 (the method as given) */
    FPTS_MIXED = 1       /* primary candidates: FP32 passes in element-local
                            coordinates, then FP64 passes from the FP32
                            result; the second search over the other
                            candidates of unsettled points is FP64; boxes,
                            codes, distances and the final residual are
                            FP64.  Line elements run FP64 throughout (their
                            map evaluation is a few dozen FLOPs) */
};

/* Setup parameters (Section 3.1).  Zero-initialise, then set fields;
 * fpts_params_default fills the paper's defaults. */
typedef struct fpts_params {
    int dim;            /* D, space dimension: 2 or 3 */
    int ref_dim;        /* D_r: dim (quad/hex mesh), 2 with dim 3 (surface
                           quads) or 1 with dim 2 or 3 (line elements,
                           Section 2 eq. eq_x_tensor_surf; OBB frame by
                           Rodrigues' rotation, Section 4.2) */
    int nodes_1d;       /* N = p + 1 GLL nodes per direction, 2..10 (p <= 9,
                           which covers every case of the paper; the Newton
                           kernels hold an element's nodes in LDS, and a hex
                           of N = 16 would need 96 KiB per wavefront);
                           FPTS_EINVAL beyond */
    int hash_n;         /* N_L cells per direction of the local map; 0 picks
                           the smallest n with n^D >= n_elem (Section 3.1.3) */
    int64_t n_elem;     /* number of elements, >= 1 */
    double bbox_tol;    /* box expansion, fraction of the extent added in
                           total (Section 3.1.1 default 0.1) */
    double surf_eps_d;  /* manifold (surface and line) INTERIOR threshold on
                           the squared distance (Section 4.4 default 1e-10) */
    int max_iter;       /* Newton passes per candidate (Section 3.2.1: 50) */
    double newton_tol;  /* stop when ||dr||_inf < newton_tol (1e-10) */
    int mixed_max_iter; /* FPTS_MIXED: FP32 passes per candidate at most */
    double mixed_tol;   /* FPTS_MIXED: the FP32 phase ends when
                           ||dr||_inf < mixed_tol (default 1e-3); the FP64
                           phase then runs the full iteration to newton_tol,
                           so this trades FP32 passes against FP64 passes
                           only.  At 1e-3 the FP32 phase takes about two
                           evaluations and the FP64 phase two (quadratic
                           convergence from ~1e-6) */
} fpts_params;

typedef struct fpts_mesh fpts_mesh;

/* Fill p with the paper's defaults for (dim, ref_dim, nodes_1d, n_elem). */
void fpts_params_default(fpts_params *p, int dim, int ref_dim, int nodes_1d,
                         int64_t n_elem);

/* Setup (Section 3.1, 4.1-4.3).  h_nodes: host array
 * [n_elem][dim][nodes_1d^ref_dim] of node coordinates, the first reference
 * index fastest (node (i,j,k) at i + N j + N^2 k).  Builds the basis and
 * bound tables, every element's axis-aligned and oriented bounding box and
 * the local Cartesian map on the host, then copies nodes, boxes and map to
 * the current HIP device on `stream` and waits for the copies.  The caller
 * keeps ownership of h_nodes.  On success *out receives a handle to release
 * with fpts_destroy.  FPTS_EINVAL for bad params, FPTS_ENOMEM, FPTS_EDEVICE. */
int fpts_setup(const fpts_params *p, const double *h_nodes, void *stream,
               fpts_mesh **out);

/* Release every host and device resource of the mesh (synchronises the
 * device first).  NULL is accepted. */
int fpts_destroy(fpts_mesh *m);

/* Move the mesh: d_nodes [n_elem][dim][nodes_1d^ref_dim] (device memory,
 * the layout of fpts_setup; may be the caller's or any buffer) become the
 * mesh's nodes, and everything fpts_setup derives from them -- element
 * AABB and OBB (Sections 3.1.1, 3.1.2, 4.1, 4.2), centres and the local
 * map (Section 3.1.3) -- is recomputed on the device, for meshes that move
 * between searches (the r-adaptivity and tangential-relaxation uses of
 * Section 6).  Element count, nodes_1d, parameters and the map resolution
 * N_L stay.  The results equal those of fpts_setup on the same nodes bit
 * for bit.  Synchronises `stream` (the map size is read back); workspace
 * sizes may grow, so query them again.  FPTS_EINVAL (null arguments, or
 * nodes whose boxes are not finite), FPTS_ENOMEM, FPTS_EDEVICE; after an
 * error the mesh must be destroyed. */
int fpts_update_nodes(fpts_mesh *m, const double *d_nodes, void *stream);

/* Bytes of device workspace fpts_find needs for n points (an upper bound
 * that assumes every point hits the largest cell of the local map), or 0
 * when n is out of range. */
size_t fpts_find_workspace_size(const fpts_mesh *m, int64_t n);

/* Find (Section 3.2, 3.2.1, 4.4): computational coordinates of n points.
 *   d_pts   [dim][n]     query coordinates (SoA)
 *   d_code  [n]  int32   FPTS_INTERIOR / FPTS_BORDER / FPTS_NOT_FOUND
 *   d_elem  [n]  int32   element id, -1 when NOT_FOUND
 *   d_r     [ref_dim][n] reference coordinates r* (0 when NOT_FOUND)
 *   d_dist  [n]          ||x* - x(r*)||_2 (+inf when NOT_FOUND)
 *   precision            FPTS_FP64 or FPTS_MIXED
 *   d_ws, ws_bytes       device workspace of at least
 *                        fpts_find_workspace_size(m, n) bytes, 256-byte
 *                        aligned; its contents need no initialisation
 * Candidates of a point are the elements of its cell whose boxes contain it;
 * each is searched with trust-region Newton; the lowest-id INTERIOR
 * candidate wins, else the one at the smallest distance (lowest id on ties).
 * n == 0 is a no-op.  FPTS_EINVAL on null pointers, n < 0, n above 2^31-1,
 * or a workspace that is too small. */
int fpts_find(fpts_mesh *m, int64_t n, const double *d_pts, int32_t *d_code,
              int32_t *d_elem, double *d_r, double *d_dist, int precision,
              void *d_ws, size_t ws_bytes, void *stream);

/* Bytes of device workspace fpts_eval needs for n points. */
size_t fpts_eval_workspace_size(const fpts_mesh *m, int64_t n);

/* Interpolate (Section 3.3, eq. eq_u_tensor with the geometry's N):
 * out[f][p] = sum over element nodes of field[f][elem[p]][node] times the
 * tensor Lagrange bases at r[p], for n_fields fields given as
 *   d_field [n_fields][n_elem][nodes_1d^ref_dim],
 * from the outputs of fpts_find (d_code, d_elem, d_r as documented there).
 * NOT_FOUND points get NaN.  Points are grouped by element on the device so
 * that each element's nodal values are read once.  FPTS_EINVAL on null
 * pointers, n_fields < 1, bad n or a too small workspace. */
int fpts_eval(fpts_mesh *m, int64_t n, const int32_t *d_code,
              const int32_t *d_elem, const double *d_r, int n_fields,
              const double *d_field, double *d_out, void *d_ws,
              size_t ws_bytes, void *stream);

/* Interpolate a field whose order differs from the geometry's (Section 2,
 * eq. eq_u_tensor, where the field has its own N-tilde nodes per direction):
 * as fpts_eval, with d_field [n_fields][n_elem][field_nodes_1d^ref_dim] of
 * nodal values at the field_nodes_1d GLL nodes per reference direction
 * (first index fastest), 2 <= field_nodes_1d <= 10.  The reference
 * coordinates r* from fpts_find are the same for every field order.
 * fpts_eval is this call with field_nodes_1d = nodes_1d.  Workspace:
 * fpts_eval_workspace_size.  FPTS_EINVAL as fpts_eval, and for
 * field_nodes_1d out of range. */
int fpts_eval_order(fpts_mesh *m, int64_t n, const int32_t *d_code, const int32_t *d_elem,
                    const double *d_r, int n_fields, int field_nodes_1d, const double *d_field,
                    double *d_out, void *d_ws, size_t ws_bytes, void *stream);

/* Bytes of device workspace fpts_find_eval needs for n points, or 0 when n
 * is out of range. */
size_t fpts_find_eval_workspace_size(const fpts_mesh *m, int64_t n);

/* Find and Interpolate in one call: the outputs of fpts_find (d_code,
 * d_elem, d_r, d_dist) and of fpts_eval_order (d_out [n_fields][n] for
 * d_field [n_fields][n_elem][field_nodes_1d^ref_dim]), bit for bit the
 * same as the two calls in a row.  The points whose primary candidate
 * settled them -- INTERIOR at least 1e-9 inside its reference box, almost
 * all interior points -- are interpolated straight from Find's own element
 * buckets, with r taken in bucket order from the workspace (no second
 * binning, no gather of r); the rest go through the binning of fpts_eval.
 * d_ws: at least fpts_find_eval_workspace_size(m, n) bytes, 256-byte
 * aligned.  FPTS_EINVAL as fpts_find and fpts_eval_order. */
int fpts_find_eval(fpts_mesh *m, int64_t n, const double *d_pts, int32_t *d_code,
                   int32_t *d_elem, double *d_r, double *d_dist, int precision, int n_fields,
                   int field_nodes_1d, const double *d_field, double *d_out, void *d_ws,
                   size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * as fpts_find_eval, with the workspace taken from a fixed array the library
 * holds on each device until the process ends (FPTS_NOALLOC_SCRATCH_BYTES
 * bytes; its address is looked up when the first mesh is set up on that
 * device).  The call allocates nothing.  It returns FPTS_ENOMEM, without
 * doing anything, when fpts_find_eval_workspace_size(m, n) exceeds
 * FPTS_NOALLOC_SCRATCH_BYTES (about 265 bytes per point plus the
 * mesh-sized arrays: some 2.0 million points on a 48^3 mesh with N = 8).
 * Every call on one device shares that device's
 * array: calls that overlap on one device -- on different streams, or
 * from different threads -- race and corrupt each other's results; they
 * must be ordered (one stream, or events).  The array keeps the last call's
 * contents; each call clears what it needs itself.  Other arguments and
 * errors as fpts_find_eval. */
#define FPTS_NOALLOC_SCRATCH_BYTES ((size_t)512 << 20)
int fpts_find_eval_noalloc(fpts_mesh *m, int64_t n, const double *d_pts, int32_t *d_code,
                           int32_t *d_elem, double *d_r, double *d_dist, int precision,
                           int n_fields, int field_nodes_1d, const double *d_field,
                           double *d_out, void *stream);

/* Counters of the last fpts_find that used workspace d_ws (read back with a
 * device-to-host copy on `stream`, which is synchronised) for one Newton
 * launch: pass 1 = primary candidates, 2 = the other candidates of points the
 * primary did not settle, 3 = the face passes of primary pairs (a pair whose
 * next pass needs second derivatives, eq. eq_newton_hessian, leaves the
 * primary kernel and resumes there, many such pairs to a wavefront), 0 = all
 * summed.  Passes and evaluations of a pair that moved to the face kernel
 * are counted where they ran; its pair is counted once, in pass 1.  A sweep
 * is one evaluation of the map by a whole wavefront at up to 16 pairs at
 * once, so evals / (16 sweeps) is the fraction of busy pair slots.
 * FPTS_EINVAL for another pass. */
typedef struct fpts_find_stats {
    int64_t pairs;          /* (point, element) pairs searched */
    int64_t passes;         /* FP64 Newton passes */
    int64_t evals;          /* FP64 map evaluations, initial ones included */
    int64_t evals_h2;       /* of which needed second derivatives */
    int64_t passes_fp32;    /* FP32 passes of mixed mode */
    int64_t evals_fp32;     /* FP32 map evaluations of mixed mode */
    int64_t evals_h2_exec;  /* FP64 evaluations computed with second
                               derivatives because a lane of the wavefront
                               needed them */
    int64_t sweeps;         /* FP64 first-derivative sweeps */
    int64_t sweeps_h2;      /* FP64 second-derivative sweeps */
    int64_t sweeps_fp32;    /* FP32 sweeps of mixed mode (both kinds) */
    int64_t overflow_points;  /* unsettled points whose other candidates did
                                 not fit the workspace's slots and were
                                 searched one point per wavefront (any
                                 pass) */
    int64_t evals_fp32_node;  /* of evals_fp32: evaluations at a start that
                                 is a GLL node, taken from the element's
                                 nodes and differentiation matrix rows
                                 without a sweep */
    int64_t parked_pairs;   /* primary pairs that reached a face in the FP64
                               primary kernel and went on in the face kernel
                               (any pass) */
    int64_t listed_points;  /* points left open by their primary result
                               whose other candidates were searched (any
                               pass) */
} fpts_find_stats;

int fpts_find_stats_get(const fpts_mesh *m, int64_t n, const void *d_ws,
                        int pass, fpts_find_stats *out, void *stream);

/* Kernel timing with HIP events recorded on the caller's stream around
 * each group of kernels of fpts_find / fpts_eval: locate (point binning,
 * candidate search and the scans), nearest (the nearest-node start of the
 * primary pass), newton (the trust-region Newton kernel of the primary pass
 * alone), select (start, Newton and selection over the other candidates of
 * unsettled points), eval_bin and eval (point binning and interpolation),
 * advance (the particle update of fpts_lpt_step, fpts_lpt.h), face (the
 * face passes of primary pairs and their binning).  Sums over
 * the calls since profiling was enabled.  Meant for one stream at a time. */
typedef struct fpts_kernel_times {
    double locate_ms;
    double nearest_ms;
    double newton_ms;
    double select_ms;
    double eval_bin_ms;
    double eval_ms;
    double advance_ms;
    double face_ms;         /* the parked face passes of the primary
                               candidates, with their binning */
    int64_t find_calls;
    int64_t eval_calls;
    int64_t lpt_calls;
} fpts_kernel_times;

/* enable != 0 starts recording (clearing earlier records); 0 stops. */
int fpts_profile(fpts_mesh *m, int enable);

/* Wait for the recorded events, return the sums and clear the records. */
int fpts_profile_read(fpts_mesh *m, fpts_kernel_times *out);

/* Read-only views of setup products, for tests and tools: copies to host
 * arrays sized [n_elem][dim][2] (AABB lo/hi), [n_elem][dim][dim] (OBB
 * inverse transform) and [n_elem][dim] (OBB centre).  Any pointer may be
 * NULL. */
int fpts_get_boxes(const fpts_mesh *m, double *h_aabb, double *h_obb_A,
                   double *h_obb_c);

/* Local map description: h_lo[dim], h_hi[dim], h_delta[dim]; returns N_L in
 * *hash_n, cell list entries in *nnz and the largest cell in *max_cell. */
int fpts_get_hash(const fpts_mesh *m, double *h_lo, double *h_hi,
                  double *h_delta, int *hash_n, int64_t *nnz, int *max_cell);

/* Cell lists of the local map (Section 3.1.3): h_cell_off[N_L^dim + 1]
 * (offsets into h_cell_el, cell (i, j, k) at i + N_L (j + N_L k)) and
 * h_cell_el[nnz] (element ids, ascending within a cell), copied to host
 * arrays sized by fpts_get_hash.  Either pointer may be NULL. */
int fpts_get_cells(const fpts_mesh *m, int32_t *h_cell_off, int32_t *h_cell_el);

/* Text of a status code. */
const char *fpts_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* FPTS_H */
