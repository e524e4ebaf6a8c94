/*
 * fpts_serve -- a request loop over resident meshes (fpts.h) on one GPU.
 *
 * Requests (find + eval of one point set against one resident mesh) are
 * queued by fpts_server_submit and served by a worker thread: requests are
 * admitted in arrival order while their device workspace fits in the
 * server's memory budget and a stream is free; requests for the same mesh
 * that are admitted together are concatenated into one batch (one
 * fpts_find_eval call, or fpts_find for a mesh without a field), and batches
 * on different streams overlap on the device.  Requests that arrive while
 * others run are admitted as soon as
 * a stream and memory free up (continuous batching).  Per-point results do
 * not depend on the batch a point travels in: each request's outputs are
 * bit-identical alone and in the mix.
 *
 * The paper's repeated Find + Interpolate of a moving point cloud (its
 * Lagrangian particle tracking loop, Section 6.7) is the use this serves;
 * the serving policy itself is not part of the paper.
 *
 * All d_* buffers are caller-owned device memory that must stay valid until
 * the request is done.  Status codes are those of fpts.h.
 */
#ifndef FPTS_SERVE_H
#define FPTS_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "fpts.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fpts_server fpts_server;

/* Request states reported by fpts_server_poll. */
enum {
    FPTS_REQ_QUEUED = 0,
    FPTS_REQ_RUNNING = 1,
    FPTS_REQ_DONE = 2,
    FPTS_REQ_FAILED = 3
};

/* Create a server on the current HIP device.  budget_bytes: device memory
 * the server allocates once and carves into request workspaces (>= 1 MiB);
 * n_streams: concurrent batches (1..16); max_batch_points: upper bound on the
 * points of one concatenated batch (>= 1).  FPTS_EINVAL, FPTS_ENOMEM,
 * FPTS_EDEVICE. */
int fpts_server_create(size_t budget_bytes, int n_streams, int64_t max_batch_points,
                       fpts_server **out);

/* Drain all work, stop the worker, release streams and the pool. */
int fpts_server_destroy(fpts_server *s);

/* Make a mesh resident for the server: fields d_field [n_fields][n_elem]
 * [nodes_1d^ref_dim] on the device (n_fields may be 0: find only).  The
 * server does not own the mesh or the fields.  *mesh_id receives its
 * index. */
int fpts_server_add_mesh(fpts_server *s, fpts_mesh *m, int n_fields, const double *d_field,
                         int *mesh_id);

/* Queue a request: n points d_pts [dim][n]; outputs as in fpts_find plus
 * d_out [n_fields][n] for the mesh's fields (may be NULL when the mesh has
 * no fields).  stream: the caller's HIP stream (NULL: the null stream) on
 * which the points are, or are being, written: the request's work waits for
 * everything queued on it before this call, so points produced by
 * asynchronous kernels or copies may be submitted at once.  The submission
 * time is taken on entry.  Returns immediately with *req_id.  FPTS_ENOMEM
 * when the request alone can never fit the budget; FPTS_EINVAL on bad
 * arguments; FPTS_EDEVICE when the readiness event cannot be recorded. */
int fpts_server_submit(fpts_server *s, int mesh_id, int64_t n, const double *d_pts,
                       int32_t *d_code, int32_t *d_elem, double *d_r, double *d_dist,
                       double *d_out, int precision, void *stream, int64_t *req_id);

/* State of a request and its times in microseconds since the server was
 * created: submitted, launched, completed on the device (HIP events). */
int fpts_server_poll(fpts_server *s, int64_t req_id, int *state, double *t_submit_us,
                     double *t_start_us, double *t_done_us);

/* Block until the request is done (or failed). */
int fpts_server_wait(fpts_server *s, int64_t req_id);

/* Block until every submitted request is done. */
int fpts_server_drain(fpts_server *s);

typedef struct fpts_server_stats {
    int64_t submitted, completed, failed, batches, points;
    int64_t max_in_flight;      /* most batches running at once */
    int64_t max_batch_requests; /* most requests in one batch */
    size_t peak_bytes;          /* most pool bytes in use at once */
    size_t budget_bytes;
} fpts_server_stats;

int fpts_server_stats_get(fpts_server *s, fpts_server_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* FPTS_SERVE_H */
