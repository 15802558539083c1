/*
 * psr.h -- C ABI of the MI355X (gfx950) differentiable Poisson solver.
 *
 * The library computes the indicator grid of Peng et al., "Shape As Points: A
 * Differentiable Poisson Solver" (NeurIPS 2021) from an oriented point cloud,
 * and the exact adjoint of that computation:
 *
 *   splat        v_d[j] = sum_i T(c_i, j/r, 1/r) n_{i,d}        (supplement Sec. A.1)
 *   solve        chi'   = IFFT( g(u) * i u.FFT(v) / (-2 pi |u|^2) )   (main Eq. 3)
 *   normalise    chi    = m / |c| * (chi' - mean_i chi'(c_i))        (main Eq. 4,
 *                         with the constraint of main Eq. 2, m = 0.5)
 *
 * Conventions (the paper leaves them open; the library and its reference agree):
 *   - periodic grid on [0,1)^3 with r vertices per axis, vertex j at j/r; point
 *     coordinates are taken mod 1; corner indices wrap mod r;
 *   - grid layout X[j0][j1][j2], row-major, j2 fastest; point column a maps to
 *     grid axis a;
 *   - u is the integer wavenumber (k for k < r/2, else k - r), sigma is in grid
 *     cells; the odd derivative factor is 0 at the Nyquist index r/2 while
 *     |u|^2 keeps (r/2)^2; chi~(0) = 0;
 *   - scale reading "B" (default): c = chi'(0,0,0) - mean, so |chi(0,0,0)| = m
 *     exactly as main Eq. 2 requires; reading "A" uses c = chi'(0,0,0) as main
 *     Eq. 4 is printed;
 *   - normals are used as given, never renormalised (supplement, outlier
 *     handling: small normals mute outliers).
 *
 * Precision: the grid work (splat, FFTs, spectral operator, gather) runs in
 * FP32 with FP32 accumulation; the mean of chi' at the points, the scale and
 * the backward reductions sum G and sum G*chi are accumulated in FP64.
 *
 * Memory: every pointer argument is DEVICE memory owned by the caller unless
 * stated otherwise. Grid-sized scratch comes in through `workspace` (size from
 * psr_workspace_bytes) and the per-solve state that backward needs lives in
 * `saved` (size from psr_saved_bytes), both owned by the caller, so a solve's
 * state lives exactly as long as the caller keeps its buffers and no free
 * call is needed. The library allocates only per context: its twiddle tables
 * at psr_ctx_create and one point-source table per (res, sigma) at the first
 * backward of that size (or at psr_ctx_prepare). Buffers must be 256-byte
 * aligned.
 *
 * Asynchrony: psr_forward, psr_backward and psr_run_batched only enqueue
 * kernels on `stream` and return. Argument errors are reported at once and
 * nothing is launched. Data-dependent errors (non-finite coordinates or normals, a zero
 * or non-finite scale) are written to a status word inside `saved`, read with
 * psr_saved_status (which synchronises the stream); the grid is then NaN.
 */
#ifndef PSR_H
#define PSR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes returned by every entry point (0 = success). */
enum {
  PSR_OK = 0,
  PSR_EINVAL = -1,        /* bad argument: NULL pointer, npoints < 1, res not a power of two in
                             [8, 512], sigma negative or non-finite, workspace too small, bad key */
  PSR_ENOMEM = -2,        /* device allocation failed (context creation only) */
  PSR_EDEGENERATE = -3,   /* scale c is zero or non-finite (e.g. all normals zero); chi is NaN */
  PSR_EDEVICE = -4,       /* a HIP runtime call failed */
  PSR_ENOTREADY = -5,     /* reserved */
  PSR_ENONFINITE = -6,    /* a point coordinate or normal component is NaN or Inf; chi is NaN */
  PSR_ETOOBIG = -7        /* the problem exceeds a fixed limit of the entry point (see its comment) */
};

#define PSR_MIN_RES 8
#define PSR_MAX_RES 512

typedef struct psr_ctx psr_ctx;

/* Library version, major*10000 + minor*100 + patch. */
int psr_version(void);

/* Human-readable text for a status code. Never NULL; the string is static. */
const char* psr_strerror(int code);

/* Create a context on HIP device `device`: uploads the FP64-built twiddle
 * tables and sets defaults (m = 0.5, reading B, timers off).
 * Returns PSR_EINVAL for a bad device, PSR_ENOMEM / PSR_EDEVICE on failure. */
int psr_ctx_create(psr_ctx** out, int device);
int psr_ctx_destroy(psr_ctx* ctx);

/* Options: "m" (target magnitude at the origin, > 0, default 0.5),
 * "reading" (0 = B, default; 1 = A), "timers" (0/1: per-stage HIP-event timing),
 * "timer_mask" (bit s set = time stage s; needs timers on; default all). */
int psr_ctx_set(psr_ctx* ctx, const char* key, double value);
int psr_ctx_get(const psr_ctx* ctx, const char* key, double* value);

/* Host-only size queries (no device calls). `with_backward` is accepted for
 * symmetry; forward and backward use the same workspace layout. */
int psr_workspace_bytes(int res, int64_t npoints, int with_backward, size_t* bytes);
int psr_saved_bytes(int res, int64_t npoints, size_t* bytes);

/* Forward solve (main Eqs. 2-4).
 *   points, normals : [npoints][3] float32, row-major. Not modified; must stay
 *                     unchanged until backward if backward is called.
 *   res             : grid vertices per axis, power of two in [8, 512].
 *   sigma           : Gaussian bandwidth in grid cells (main Eq. 3), >= 0.
 *   chi             : [res][res][res] float32 output (written in full).
 *   saved           : psr_saved_bytes(res, npoints) bytes; receives the sorted
 *                     points, the scalars mean/c/scale/chi'(0) and the status.
 *   workspace       : at least psr_workspace_bytes(res, npoints, .) bytes.
 * The call is stream-ordered and asynchronous. */
int psr_forward(psr_ctx* ctx, const float* points, const float* normals, int64_t npoints,
                int res, float sigma, float* chi, void* saved, void* workspace,
                size_t workspace_bytes, hipStream_t stream);

/* Forward solve that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc). Same arguments and result as psr_forward without
 * `saved` and `workspace`: both are carved from one static device array of
 * PSR_STATIC_SCRATCH_BYTES per GPU (64 MiB, held from library load until the
 * process ends), whose address the context takes at psr_ctx_create. The
 * call makes no hipMalloc, hipFree or other allocating call.
 *   Limit: psr_saved_bytes(res, npoints) + psr_workspace_bytes(res, npoints)
 *   must not exceed PSR_STATIC_SCRATCH_BYTES (res 128 with up to 57,036
 *   points, res 64 with up to 216,432, res 32 with up to 236,622; no res of
 *   256 or more fits); larger problems return PSR_ETOOBIG and launch nothing.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (each call re-initialises what it reads): calls that overlap on
 * one GPU (two streams, or two threads) race and must be serialised by the
 * caller. There is no backward for this call (its state is not kept), and
 * the status of the solve is not reported: a degenerate or non-finite input
 * gives a NaN grid. */
#define PSR_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int psr_forward_static(psr_ctx* ctx, const float* points, const float* normals, int64_t npoints, int res,
                       float sigma, float* chi, hipStream_t stream);

/* Backward (adjoint) of psr_forward: the gradient of a loss L(chi) with
 * respect to the oriented points that main Sec. 3.1 asks of the solver (the
 * paper differentiates Eqs. 3-4 by autograd; here the adjoint is written out:
 * transposed splat, conjugate spectral operator, transposed gather, and the
 * derivative of the Eq. 4 normalisation through mean, c and m/|c|).
 * Given dchi = dL/dchi, writes dpoints = dL/dpoints and dnormals = dL/dnormals
 * ([npoints][3] float32; either may be NULL to skip it). `chi` is the
 * forward's output and `saved` its state, both unchanged since the forward;
 * npoints/res/sigma must repeat the forward's. The saved header records the
 * forward's res and npoints: if they differ from this call's, every backward
 * kernel returns without reading the saved records or the workspace, and
 * dpoints/dnormals are filled with NaN (the call itself returns PSR_OK, as the
 * check runs on the device). The derivative of the position wrap (mod 1) is
 * taken as 1; on a cell face the derivative is the one of the cell above
 * (right derivative). */
int psr_backward(psr_ctx* ctx, int64_t npoints, int res, float sigma, const float* chi,
                 const void* saved, const float* dchi, float* dpoints, float* dnormals,
                 void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Build the backward's point-source table for (res, sigma) now, on `stream`
 * (synchronising it once), instead of on the first psr_backward or
 * psr_run_batched call with that size. The table is the response of the
 * adjoint spectral operator of main Eq. 3 to a unit source at grid vertex 0:
 * the derivative of Eq. 4 through chi'(0,0,0) puts a point source of weight
 * -Q = -sum(G chi)/c at that vertex, whose FP32 transform alongside the rest
 * of the cotangent would lose its precision when Q is large, so its effect
 * is read at the points from this table, built in FP64 and kept as float
 * ((res/2 + 1)^3 floats, 8.6 MB at 256^3) until psr_ctx_destroy. The first
 * backward at a new (res, sigma) allocates the table and a temporary build
 * buffer and synchronises its stream; later calls allocate nothing.
 * Returns PSR_EINVAL, PSR_ENOMEM or PSR_EDEVICE on failure. */
int psr_ctx_prepare(psr_ctx* ctx, int res, float sigma, hipStream_t stream);

/* Synchronises `stream`, then reads the status word written by the forward
 * on that stream into *status (PSR_OK, PSR_EDEGENERATE or PSR_ENONFINITE).
 * EDEGENERATE is the case where the scale of main Eq. 4 cannot be formed
 * (c = 0 or non-finite, so m/|c| of Eq. 2's constraint is undefined). */
int psr_saved_status(const void* saved, hipStream_t stream, int* status);

/* Synchronises `stream`, then reads the forward's FP64 scalars of main Eq. 4:
 * the mean of chi' at the points, the scale denominator c, the scale m/|c| and
 * chi'(0,0,0). Any output pointer may be NULL. */
int psr_saved_scalars(const void* saved, hipStream_t stream, double* mean, double* cscale,
                      double* scale, double* chi0);

/* One solve of a batch. Inputs/outputs as in psr_forward/psr_backward.
 * With stages = PSR_JOB_FORWARD (0): `dchi` NULL = forward only; otherwise the
 * backward runs right after the forward and writes dpoints/dnormals (either
 * may be NULL). With stages = PSR_JOB_BACKWARD: only the backward runs, from
 * the chi and saved state that an earlier forward of this job left (same
 * npoints, res, sigma; points and normals may be NULL), so that an autograd
 * caller can batch its forwards and, later, its backwards. `workspace` and
 * `saved` are per job and must not overlap between jobs. */
#define PSR_JOB_FORWARD 0
#define PSR_JOB_BACKWARD 2
typedef struct psr_job {
  const float* points;
  const float* normals;
  int64_t npoints;
  int res;
  float sigma;
  float* chi;
  void* saved;
  const float* dchi;
  float* dpoints;
  float* dnormals;
  void* workspace;
  size_t workspace_bytes;
  int32_t stages;  /* PSR_JOB_FORWARD or PSR_JOB_BACKWARD */
  int32_t reserved;
} psr_job;

/* Run `njobs` independent solves with one launch per pipeline stage for the
 * whole batch (jobs may mix resolutions, point counts and stages): the batched
 * form of psr_forward/psr_backward. Stream-ordered. */
int psr_run_batched(psr_ctx* ctx, int njobs, const psr_job* jobs, hipStream_t stream);

/* Test hooks. psr_debug_spectral runs only the spectral solve on a given
 * field v ([3][res^3] float32) and writes the unnormalised chi' ([res^3]).
 * psr_debug_splat writes the rasterised field v ([3][res^3]) for the points;
 * `saved` and `workspace` as for psr_forward. */
int psr_debug_spectral(psr_ctx* ctx, const float* v, int res, float sigma, float* chi_prime,
                       void* workspace, size_t workspace_bytes, hipStream_t stream);
int psr_debug_splat(psr_ctx* ctx, const float* points, const float* normals, int64_t npoints,
                    int res, float* v, void* saved, void* workspace, size_t workspace_bytes,
                    hipStream_t stream);

/* ------------------------------------------------------------------------
 * Slab-decomposed forward solve for large grids (16^3 to 1024^3): the
 * large-scene form of the solver (main Sec. 5: the dense grid's memory grows
 * with the cube of the resolution). It computes the same chi as psr_forward
 * (main Eqs. 2-4, same conventions and options) with the grid cut along j0
 * into `slabs` slabs of res/slabs planes. Each stage runs per slab (splat +
 * r2c along j2, FFT along j1; inverse FFT along k1, c2r along k2, gather at
 * the slab's points) or per pencil owner (FFT along j0 with the spectral
 * operator of main Eq. 3 over res/slabs values of k1), and the spectrum
 * moves between them in equal blocks, as an all-to-all between processes
 * would move it; the gather reads one halo plane of the next slab. Forward
 * only: there is no backward of this call.
 * The result does not depend on `slabs`: chi and the scalars are the same
 * bit for bit for every slab count.
 * ------------------------------------------------------------------------ */
#define PSR_SLAB_MAX_RES 1024
#define PSR_SLAB_MAX_SLABS 64

/* Scalars of the slab forward (main Eq. 4), written to device memory. */
typedef struct psr_slab_result {
  double mu;       /* mean of chi' at the points (FP64) */
  double cscale;   /* c: chi'(0,0,0) - mu (reading B) or chi'(0,0,0) (reading A) */
  double scale;    /* m / |c|; NaN when status != PSR_OK */
  double chi0;     /* chi'(0,0,0) */
  int32_t status;  /* PSR_OK, PSR_EDEGENERATE or PSR_ENONFINITE */
  int32_t flags;   /* bit 0: a non-finite coordinate or normal was seen */
} psr_slab_result;

/* Workspace bytes of the slab forward (host only). res: power of two in
 * [16, 1024]; slabs: power of two in [1, min(64, res)]; npoints may be 0 for
 * psr_slab_debug_spectral. About 48 res^2 (res/2 + 16) bytes of grid buffers
 * plus 80 bytes per point (26 GB at 1024^3). */
int psr_slab_workspace_bytes(int res, int64_t npoints, int slabs, size_t* bytes);

/* Slab forward. points, normals [npoints][3] float32; chi [res][res][res]
 * float32 output (written in full; slab g is planes [g res/slabs,
 * (g+1) res/slabs)); result: one psr_slab_result in device memory, written
 * by the last kernel (read it after synchronising the stream); workspace at
 * least psr_slab_workspace_bytes bytes, 256-byte aligned. Data-dependent
 * errors go to result->status (the grid is then NaN). Stream-ordered and
 * asynchronous; returns PSR_EINVAL for a bad argument (nothing launched) or
 * PSR_EDEVICE if a launch failed. */
int psr_slab_forward(psr_ctx* ctx, const float* points, const float* normals, int64_t npoints, int res, float sigma,
                     int slabs, float* chi, psr_slab_result* result, void* workspace, size_t workspace_bytes,
                     hipStream_t stream);

/* Test hook: the slab passes on a given field v ([3][res^3] float32) instead
 * of the splat; writes the unnormalised chi' ([res^3]) as psr_debug_spectral
 * does. workspace: psr_slab_workspace_bytes(res, 0, slabs) bytes. */
int psr_slab_debug_spectral(psr_ctx* ctx, const float* field, int res, float sigma, int slabs, float* chi_prime,
                            void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Marching Cubes on the indicator grid and its inverse-normal gradient
 * (main Sec. 3.2: the mesh of chi by Marching Cubes, Lorensen and Cline 1987;
 * main Eq. 6: dp_mesh/dchi = -n_mesh).
 *
 * The surface is the level chi = iso (main Eq. 2 makes the mean of chi at
 * the input points 0, so iso = 0 passes through them). The grid is sampled as
 * an image volume: cells (j, j+1) along each axis for j in [0, res-2], vertex
 * j at position j/res. A grid edge whose ends lie on different sides of the
 * level (inside = chi < iso) carries one mesh vertex at
 * t = (chi_a - iso)/(chi_a - chi_b) along it; its normal is the periodic
 * central-difference gradient of chi interpolated with the same t and
 * normalised (it points to chi > iso, outward). Vertices are numbered by
 * global edge id 3 * (row-major index of the edge's lower end) + axis;
 * triangles by cell (row-major), then case-table order, counter-clockwise
 * seen from outside. Faces with four crossing edges cut each inside corner
 * off on its own, so the mesh is closed and edge-manifold wherever the
 * level set stays inside the grid.
 * ------------------------------------------------------------------------ */

/* Bytes of the state buffer for a res^3 grid (host-only query): per-vertex
 * base indices (4 res^3 bytes), per-workgroup counts and a header. */
int psr_mc_state_bytes(int res, size_t* bytes);

/* Mesh of chi ([res]^3 float32, device) at the level iso. Writes up to vcap
 * vertices (verts, normals: [vcap][3] float32; edges: [vcap] int32 global
 * edge ids, may be NULL) and up to tcap triangles (tris: [tcap][3] int32
 * vertex indices); `state` (psr_mc_state_bytes, caller-owned, 256-byte
 * aligned) receives the totals and the vertex map that the backward needs.
 * Stream-ordered; the totals are read with psr_mc_counts. If a total exceeds
 * its capacity the output is truncated (triangles may then index vertices
 * beyond vcap): call again with larger buffers. */
int psr_marching_cubes(psr_ctx* ctx, const float* chi, int res, float iso, float* verts, float* normals,
                       int32_t* edges, int64_t vcap, int32_t* tris, int64_t tcap, void* state,
                       hipStream_t stream);

/* Synchronises `stream` and reads the totals of the last psr_marching_cubes
 * into *nverts and *ntris (either may be NULL); *status (may be NULL) is
 * PSR_OK, or PSR_ETOOBIG when the mesh has 2^29 vertices or more (the vertex
 * map cannot hold them; the output is then not valid). */
int psr_mc_counts(const void* state, hipStream_t stream, int64_t* nverts, int64_t* ntris, int* status);

/* Gradient of a loss through the mesh vertices back to the grid (main Eq. 6):
 * with g_v = -(dL/dp_v . n_v) for vertex v on the grid edge (a, b) at t,
 * dchi[a] += (1 - t) g_v and dchi[b] += t g_v; every grid value of dchi
 * ([res]^3 float32) is written. `chi`, `iso` and `state` are those of the
 * forward, unchanged; normals are the forward's, dverts = dL/dverts
 * ([nverts][3]); vertices at or beyond nverts contribute nothing. If `state`
 * was made for another res or iso, dchi is filled with NaN. */
int psr_marching_cubes_backward(psr_ctx* ctx, const float* chi, int res, float iso, const void* state,
                                const float* normals, const float* dverts, int64_t nverts, float* dchi,
                                hipStream_t stream);

/* ------------------------------------------------------------------------
 * The optimisation-based reconstruction loop around the solver (main Sec.
 * 3.2): points sampled on the mesh (the p_mesh of main Eq. 5), the
 * bidirectional Chamfer loss of Eq. 5 against a target cloud, and the mesh's
 * connected components for the resampling from the largest one (main Sec.
 * 3.2, "Resampling"). All arrays are device memory; vertices [n][3] float32,
 * faces [n][3] int32.
 * ------------------------------------------------------------------------ */

/* Bytes of the sampling workspace for a mesh of nfaces triangles (host only). */
int psr_mesh_sample_workspace_bytes(int64_t nfaces, size_t* bytes);

/* nsamples points uniformly by area on the mesh, from the random numbers
 * u ([nsamples][3] float32 in [0, 1), caller-drawn): u0 picks the first
 * triangle whose running (FP64) area sum exceeds u0 times the total, u1 and
 * u2 give the barycentric weights (1 - sqrt(u1), sqrt(u1)(1 - u2),
 * sqrt(u1) u2). face_weight ([nfaces] float32, may be NULL) multiplies the
 * areas (0/1 restricts the draw to a set of faces, e.g. the largest
 * component); if the weighted total is zero the samples come from the last
 * triangle. Writes points [nsamples][3], face [nsamples] (triangle index),
 * bary [nsamples][3], and, when normals is not NULL, the vertex normals
 * (vnormals) interpolated with the same weights and normalised. */
int psr_mesh_sample(psr_ctx* ctx, const float* verts, const float* vnormals, int64_t nverts, const int32_t* faces,
                    int64_t nfaces, const float* face_weight, const float* u, int64_t nsamples, float* points,
                    float* normals, int32_t* face, float* bary, void* workspace, size_t workspace_bytes,
                    hipStream_t stream);

/* dverts = dL/dverts ([nverts][3], overwritten) from dpoints = dL/dpoints of
 * the samples: each sample adds its barycentric share to its triangle's
 * three vertices (float atomics: the summation order, and so the last bits,
 * may differ between runs). */
int psr_mesh_sample_backward(psr_ctx* ctx, const int32_t* faces, int64_t nverts, const int32_t* face,
                             const float* bary, const float* dpoints, int64_t nsamples, float* dverts,
                             hipStream_t stream);

/* Bytes of the Chamfer workspace for nx samples and ny target points (host only). */
int psr_chamfer_workspace_bytes(int64_t nx, int64_t ny, size_t* bytes);

/* Bidirectional L2 Chamfer distance (main Eq. 5) between x ([nx][3]) and y
 * ([ny][3]): nn_x[i] / d_x[i] = nearest y and its squared distance, nn_y /
 * d_y the same from y to x, and, when loss is not NULL, *loss = mean(d_x) +
 * mean(d_y) (one double, device memory, FP64 sums in a fixed order). The
 * result is the brute-force one (squared FP32 distances, equal distances go
 * to the lower index): both clouds are sorted into spatial tiles and a tile
 * is skipped only when its box is farther than a distance already found.
 * A point with a NaN coordinate is nobody's neighbour; a query with one gets
 * index -1 and distance +inf. */
int psr_chamfer(psr_ctx* ctx, const float* x, int64_t nx, const float* y, int64_t ny, int32_t* nn_x, float* d_x,
                int32_t* nn_y, float* d_y, double* loss, void* workspace, size_t workspace_bytes,
                hipStream_t stream);

/* grad_x = dL/dx of the Chamfer loss from its nearest-neighbour indices:
 * 2 (x_i - y_nn_x[i]) / nx, plus 2 (x_i - y_j) / ny for every j with
 * nn_y[j] = i (float atomics for the second term). A sample without a
 * neighbour (nn_x[i] = -1) gets NaN; a target point without one adds nothing. */
int psr_chamfer_backward(psr_ctx* ctx, const float* x, int64_t nx, const float* y, int64_t ny, const int32_t* nn_x,
                         const int32_t* nn_y, float* grad_x, hipStream_t stream);

/* Bytes of the components workspace (host only). */
int psr_mesh_components_workspace_bytes(int64_t nverts, int64_t nfaces, size_t* bytes);

/* Connected components of the mesh (triangles sharing a vertex): labels
 * ([nverts] int32) = the smallest vertex index of each vertex's component;
 * when largest ([nfaces] float32) is not NULL, 1 for the triangles of the
 * component with the greatest area (ties: the lowest label), else 0.
 * Synchronises `stream` after every relaxation pass (it reads a change flag);
 * returns PSR_ENOTREADY if 256 passes did not settle the labels. */
int psr_mesh_components(psr_ctx* ctx, const float* verts, int64_t nverts, const int32_t* faces, int64_t nfaces,
                        int32_t* labels, float* largest, void* workspace, size_t workspace_bytes,
                        hipStream_t stream);

/* Bytes of the workspace of psr_opt_step (host only): the solve's workspace,
 * saved state and grids, the Marching Cubes state and a mesh of at most vcap
 * vertices and tcap triangles, the samples, the Chamfer buffers and every
 * gradient. */
int psr_opt_step_workspace_bytes(int res, int64_t npoints, int64_t ntarget, int64_t nsamples, int64_t vcap,
                                 int64_t tcap, size_t* bytes);

/* One iteration of the optimisation-based reconstruction (main Sec. 3.2,
 * Eqs. 5-6), in one call instead of one per step: the solve of (points,
 * normals) on the res^3 grid, Marching Cubes of chi = 0 (at most vcap
 * vertices, tcap triangles), nsamples points sampled by area with the
 * caller's uniform numbers u ([nsamples][3] in [0, 1)), the Chamfer loss to
 * target ([ntarget][3]), the backward through the samples, the mesh and the
 * solver's adjoint, and one Adam step with step count t >= 1 (learning rate
 * lr, beta1, beta2, eps; first and second moments m_*, v_* of points and
 * normals, [npoints][3] float32, updated in place) on the points, which are
 * then wrapped into [0, 1) (the periodic domain), and on the normals.
 * *loss (device double) receives the Chamfer loss; mesh_counts (host,
 * int64_t[2], may be NULL) the mesh's vertices and triangles. The same
 * kernels as the separate calls, in the same order. Synchronises the stream
 * once, to read the mesh size. Returns PSR_ETOOBIG with points, normals and
 * moments untouched when the mesh exceeds vcap or tcap (mesh_counts then
 * holds the sizes needed), PSR_EDEGENERATE when the mesh is empty. Calls
 * that overlap on one workspace race. */
int psr_opt_step(psr_ctx* ctx, float* points, float* normals, int64_t npoints, float* m_points, float* v_points,
                 float* m_normals, float* v_normals, int64_t t, float lr, float beta1, float beta2, float eps,
                 const float* target, int64_t ntarget, const float* u, int64_t nsamples, int res, float sigma,
                 int64_t vcap, int64_t tcap, double* loss, int64_t* mesh_counts, void* workspace,
                 size_t workspace_bytes, hipStream_t stream);

/* Test hook (host only): the case table the kernels use. ntri[256]: triangles
 * per sign pattern (bit k = corner k inside, corner k at offset (k&1,
 * (k>>1)&1, k>>2)); edges[256][15]: their local edge ids, edge 4a + u + 2v
 * along axis a from the corner whose other two coordinates are (u, v). */
int psr_mc_case_table(int8_t* ntri, int8_t* edges);

/* Stage timers (enabled with psr_ctx_set(ctx, "timers", 1)). Synchronises all
 * recorded events and returns, per stage id in [0, n), the summed duration in
 * milliseconds and the number of launches timed; psr_stage_name gives the id's
 * name. psr_ctx_reset_timers clears the sums. */
int psr_ctx_stage_times(psr_ctx* ctx, double* ms, int64_t* counts, int n);
int psr_ctx_reset_timers(psr_ctx* ctx);
const char* psr_stage_name(int stage);
int psr_num_stages(void);

#ifdef __cplusplus
}
#endif
#endif /* PSR_H */
