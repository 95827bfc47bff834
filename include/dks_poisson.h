/*
 * dks_poisson.h -- C ABI of the MI355X free-space particle-mesh Poisson solver.
 *
 * The library computes the open-boundary potential of a charge distribution
 * by Hockney's method as the paper states it (section "FFT Based
 * Particle-Mesh Solver"): charge is assigned to a regular 3-D mesh by
 * cloud-in-cell, the mesh is zero-padded to twice its size per axis, the
 * potential is the discrete convolution with the Green's function of the
 * free-space Poisson equation (the brute-force sum equation, computed as the
 * Hadamard product of forward FFTs followed by an inverse FFT), the field is
 * the negative central-difference gradient, and it is interpolated back to the
 * particles by cloud-in-cell.  The Green's function is the cell-integrated
 * 1/r kernel, computed in FP64 on the device.
 *
 * Conventions shared by every entry point
 *  - Memory: the caller owns every buffer, including the workspace, and
 *    allocates it (the paper's DKS leaves memory management to the user,
 *    section "DKS" and its usage example).  Pointers marked "device" must be
 *    device memory of the current HIP device; the library never frees them.
 *  - Layout: meshes are C-contiguous [nz][ny][nx] (x fastest); a mesh vector
 *    field is [3][nz][ny][nx] ordered (x, y, z) components.  Particles are
 *    structure-of-arrays: separate x, y, z arrays of np elements.
 *  - Types: every array has the plan's dtype (float for DKS_F32, double for
 *    DKS_F64).  Every host scalar is double.  Units are SI (m, C, V, V/m).
 *  - Streams: every device operation is enqueued asynchronously on the
 *    caller's stream (NULL = the default stream), with no host
 *    synchronisation, so a solve can be captured into a HIP graph.  The
 *    exceptions are dks_poisson_geometry, which synchronises the stream, and
 *    the host-resident solves, whose copies run on streams of the plan.
 *  - Mesh: node (i, j, k) sits at origin + (i hx, j hy, k hz).  An
 *    explicit-h plan is centred at 0 unless dks_poisson_set_origin moves it.
 *    A fitted plan (hx = hy = hz = 0) re-fits a cubic mesh to the particles
 *    of every particle solve: h = max_d extent_d / (n_d - 3), origin centring
 *    the particles' bounding box (at least one empty node on each side); with
 *    no particles or a zero extent, h = 1 m.
 *  - Particles outside the mesh (a cell coordinate (x - x0) * (1/h), taken
 *    in the plan's dtype, below 0 or above n - 1 on any axis) deposit
 *    nothing, receive E = 0 and are counted.
 *  - Errors: every entry point returns a dks_status.  Arguments are checked
 *    on the host before any device work; no C++ exception crosses the ABI.
 *    HIP failures are reported as DKS_EHIP.  A plan is not thread-safe;
 *    distinct plans may run concurrently on distinct streams.
 */
#ifndef DKS_POISSON_H
#define DKS_POISSON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DKS_OK = 0,
  DKS_EINVAL = -1,        /* bad argument: null pointer, size or spacing out of range */
  DKS_EUNSUPPORTED = -2,  /* a doubled extent 2n is not of the form 2^a 3^b, or too large */
  DKS_ENOMEM = -3,        /* host allocation failed */
  DKS_EHIP = -4,          /* a HIP runtime call or kernel launch failed */
  DKS_EWORKSPACE = -5,    /* workspace missing, too small or misaligned */
  DKS_ESTATE = -6         /* call out of order (e.g. solve before prepare) */
} dks_status;

typedef enum { DKS_F32 = 0, DKS_F64 = 1 } dks_dtype;

/* Kernel of the convolution (section "FFT Based Particle-Mesh Solver"):
 *   DKS_GREEN_INTEGRATED : 1/r integrated over one mesh cell (default);
 *   DKS_GREEN_POINT      : the brute-force equation's point kernel 1/r at the
 *                          node offsets times the cell volume, with the cell
 *                          integral at the singular zero offset. */
typedef enum { DKS_GREEN_INTEGRATED = 0, DKS_GREEN_POINT = 1 } dks_green;

/* Charge assignment and field interpolation (the NGP / CIC / TSI box of the
 * OPAL structure figure):
 *   DKS_ASSIGN_CIC : cloud in cell, 8 nodes, linear weights (default);
 *   DKS_ASSIGN_NGP : nearest grid point, floor(s + 1/2);
 *   DKS_ASSIGN_TSC : triangular-shaped cloud, 27 nodes, quadratic weights
 *                    ((1/2 - d)^2 / 2, 3/4 - d^2, (1/2 + d)^2 / 2) around the
 *                    nearest node, d = s - nearest.
 * s = (x - x0) / h in node units.  A particle is outside the mesh when some
 * s_d is outside [0, n_d - 1] or, for TSC, its nearest node is outside
 * [1, n_d - 2] (the stencil must lie on the mesh). */
typedef enum { DKS_ASSIGN_CIC = 0, DKS_ASSIGN_NGP = 1, DKS_ASSIGN_TSC = 2 } dks_assign;

typedef struct dks_poisson_plan_s* dks_poisson_plan_t;

/* A hipStream_t passed as an opaque pointer (NULL = default stream). */
typedef void* dks_stream_t;

/* Create a plan for an nx x ny x nz node mesh (section "FFT Based
 * Particle-Mesh Solver": the M_x x M_y x M_z mesh, solved on the doubled
 * 2M grid).
 *   nx, ny, nz : nodes per axis, each >= 2 (>= 4 for a fitted plan); each
 *                2 n_d must factor as 2^a 3^b and be <= 4096.
 *   hx, hy, hz : cell sizes in metres, all > 0 (explicit mesh), or all
 *                exactly 0 (particle-fitted cubic mesh).
 *   dtype      : arithmetic type of the bulk path and of every array.
 *   out        : receives the plan handle (host memory owned by the library
 *                until dks_poisson_destroy).
 * Host-only; touches no device. */
dks_status dks_poisson_plan(int nx, int ny, int nz, double hx, double hy, double hz,
                            dks_dtype dtype, dks_poisson_plan_t* out);

/* Move an explicit-h mesh: node (0,0,0) at (x0, y0, z0) metres (the mesh
 * the solver section places over the bunch; here its position is the
 * caller's choice instead of a fit).  Takes effect from the next solve.
 * Host-only.  DKS_EINVAL for a non-finite value, DKS_ESTATE on a fitted
 * plan. */
dks_status dks_poisson_set_origin(dks_poisson_plan_t plan, double x0, double y0, double z0);

/* Select the convolution kernel and the assignment scheme (defaults:
 * integrated kernel, CIC).  Host-only.  Changing the kernel invalidates the
 * cached spectrum: solves return DKS_ESTATE until dks_poisson_prepare runs
 * again.  DKS_EINVAL for an unknown value. */
dks_status dks_poisson_set_scheme(dks_poisson_plan_t plan, dks_green green, dks_assign assign);

/* Order-independent deposit (default off): on = 1 makes the charge
 * assignment (the deposit, in the paper's OPAL structure "NGP, CIC, TSI",
 * section "The DKS Implementation of the Poisson Solver") independent of the
 * order of the particles and of the scheduling of the work, so that a solve
 * repeated on the same particles, in any order, gives bitwise the same phi
 * and, particle for particle, the same field.  Each work item's fixed-point
 * sum is added to an exact integer total per mesh node (64 bits in FP32,
 * 128 in FP64) kept in the plan's workspace, and the weights are formed from
 * the totals once; the default adds the items' sums in floating point, whose
 * rounding depends on the order.  Costs one more pass over the mesh.
 * Host-only; takes effect from the next solve.  DKS_EINVAL for on other than
 * 0 or 1. */
dks_status dks_poisson_set_deterministic(dks_poisson_plan_t plan, int on);

/* Bytes of device workspace the plan needs: its resident state (Green's
 * spectrum octant, twiddle tables, geometry block) plus the scratch of one
 * solve.  The caller allocates it (section "DKS": memory management is left
 * to the user, as in its allocate / write / call / read / free example).
 * Alignment required: 256 bytes.  Host-only; DKS_EINVAL for NULL. */
dks_status dks_poisson_workspace_bytes(dks_poisson_plan_t plan, size_t* bytes);

/* Bytes of per-element scratch a batched solve needs for `batch` elements
 * of at most max_np particles each, on top of the plan workspace: each
 * element's mesh intermediates and its binned particle records.  Caller-
 * allocated like every buffer (section "DKS": memory management is the
 * user's).  Host-only; DKS_EINVAL for batch outside 1..16, a negative or too
 * large max_np, or NULL. */
dks_status dks_poisson_batch_scratch_bytes(dks_poisson_plan_t plan, int batch, int64_t max_np,
                                           size_t* bytes);

/* Particle solves and the deposit group the particles by mesh tile before
 * depositing (so that the CIC charge assignment of the OPAL structure figure
 * accumulates in on-chip memory rather than by contended device-wide
 * atomics) and need a caller-owned device scratch of
 * dks_poisson_particle_scratch_bytes(np) bytes for np particles (16 bytes per
 * particle in FP32, 28 in FP64: the binned (x, y, z) record and the inverse
 * permutation, each rounded up to 256), attached with
 * dks_poisson_set_particle_scratch (256-byte aligned; NULL with 0 bytes
 * detaches).  A solve of more particles than the attached scratch holds
 * returns DKS_EWORKSPACE.  np must be at most 2^32 - 2^20. */
dks_status dks_poisson_particle_scratch_bytes(dks_poisson_plan_t plan, int64_t np, size_t* bytes);
dks_status dks_poisson_set_particle_scratch(dks_poisson_plan_t plan, void* scratch, size_t bytes);

/* Attach caller-owned device workspace (at least dks_poisson_workspace_bytes,
 * 256-byte aligned).  The plan keeps the pointer; the caller keeps it alive
 * and must call dks_poisson_prepare again after attaching a new one. */
dks_status dks_poisson_set_workspace(dks_poisson_plan_t plan, void* workspace, size_t bytes);

/* Build the resident state on the device, on `stream`: the FP64 twiddle
 * tables (rounded to the dtype) and the Green's function spectrum.  The
 * spectrum is the DFT over the doubled grid of the cell-integrated 1/r kernel
 * (the G of the convolution-solution equation, integrated over a cell; FFT of
 * G in the paper's sequence diagram), evaluated and transformed in FP64, with
 * the 1/(Nx Ny Nz) inverse-transform factor folded in, then rounded to the
 * dtype.  Because the kernel is even, its spectrum is real and even, and only
 * the octant [0..nx] x [0..ny] x [0..nz] is stored.  Must precede any solve;
 * a fitted plan computes it once for h = 1 m and scales it by h^2 per solve. */
dks_status dks_poisson_prepare(dks_poisson_plan_t plan, dks_stream_t stream);

/* Potential (and field) of a mesh charge density (the brute-force sum
 * equation and its FFT form; E = -grad phi by central differences, the
 * D-operator of the OPAL structure figure).  Explicit-h plans only
 * (DKS_ESTATE on a fitted plan).
 *   rho    : device [nz][ny][nx], C/m^3, read only.
 *   phi    : device [nz][ny][nx], volts, written; may be NULL.
 *   E_mesh : device [3][nz][ny][nx], V/m, written; may be NULL.
 * At least one of phi, E_mesh must be non-NULL. */
dks_status dks_poisson_solve_rho(dks_poisson_plan_t plan, const void* rho, void* phi,
                                 void* E_mesh, dks_stream_t stream);

/* One full particle step (section "FFT Based Particle-Mesh Solver" and the
 * OPAL structure figure): (fit the mesh to the bunch,) CIC deposit of the
 * charge, free-space potential by the doubled-grid FFT convolution with the
 * Green's function, central-difference field, CIC gather back to the
 * particles.  Needs the attached particle scratch (DKS_EWORKSPACE without
 * room for np particles), the workspace and a prepared spectrum
 * (DKS_ESTATE otherwise).
 *   x, y, z    : device [np] particle positions in metres, read only.
 *   np         : number of particles, 0 <= np <= 2^32 - 2^20.
 *   q          : charge of each particle in coulombs.
 *   Ex, Ey, Ez : device [np] field at the particles, V/m, written (np > 0).
 *   phi        : device [nz][ny][nx] mesh potential, volts; may be NULL.
 *   n_outside  : device int64 counter of particles outside the mesh, written
 *                (not accumulated); may be NULL. */
dks_status dks_poisson_solve_particles(dks_poisson_plan_t plan, const void* x, const void* y,
                                       const void* z, int64_t np, double q, void* Ex, void* Ey,
                                       void* Ez, void* phi, int64_t* n_outside,
                                       dks_stream_t stream);

/* The particle step for a caller that keeps its particles on the device
 * and lets the solver order them (the paper's particle-matter offload keeps
 * its particles resident on the device between steps and sorts them there,
 * section "The DKS Implementation of the Particle Matter Interaction
 * Model"): the same step as dks_poisson_solve_particles, but the particles
 * come back in the order the step binned them, 16^3-cell tile by tile of
 * this step's mesh (particles outside the mesh last), instead of in their
 * input order.
 *   x, y, z             : device [np] positions, read only.
 *   x_out, y_out, z_out : device [np], written with the same positions in
 *                         the binned order (they hold the binned particles
 *                         during the step); must not overlap x, y, z, the
 *                         field outputs or each other (DKS_EINVAL).  A
 *                         caller keeping its particles resident alternates
 *                         between two sets of position arrays.
 *   Ex, Ey, Ez          : device [np] field at the particles in the binned
 *                         order.
 *   new_index           : device uint32 [np] or NULL (then the step writes
 *                         no permutation); new_index[i] receives the new
 *                         position of the particle that was at index i, so
 *                         the caller can move its other per-particle arrays
 *                         the same way (a[new_index[i]] = a_before[i]).  It
 *                         must not overlap the other arrays (DKS_EINVAL).
 * Other arguments, limits and errors as dks_poisson_solve_particles.  The
 * step needs no reordering pass of its own (the field is written in the
 * binned order), and particles that arrive in the previous step's order
 * are binned with long runs of consecutive writes. */
dks_status dks_poisson_solve_particles_sorted(dks_poisson_plan_t plan, const void* x, const void* y,
                                              const void* z, int64_t np, double q, void* x_out,
                                              void* y_out, void* z_out, void* Ex, void* Ey, void* Ez,
                                              void* phi, uint32_t* new_index, int64_t* n_outside,
                                              dks_stream_t stream);

/* One element of a batched particle solve.  The table of elements lives in
 * device memory and is read by the kernels when they run, so a HIP graph
 * captured over dks_poisson_solve_particles_batched can be replayed for new
 * particle sets by rewriting the table (same table address, same batch).
 * Every field is 8 bytes; the struct is 80 bytes. */
typedef struct {
  const void* x;         /* device [np] positions, metres */
  const void* y;
  const void* z;
  void* Ex;              /* device [np] field at the particles, V/m, written */
  void* Ey;
  void* Ez;
  void* phi;             /* device [nz][ny][nx] potential, volts, or NULL */
  int64_t* n_outside;    /* device counter of particles outside the mesh, or NULL */
  int64_t np;            /* particle count; clamped to [0, max_np] */
  double q;              /* charge of each particle, coulombs */
} dks_particle_set;

/* The particle step for `batch` independent particle sets of the plan's
 * shape and dtype (the many solver clients the paper's DKS implementation of
 * the Poisson solver lets share one GPU, section "The DKS Implementation of
 * the Poisson Solver"), each kernel launched once over the whole batch (the
 * batch index is part of the grid).  On a fitted plan every element gets its own
 * mesh fit, and the cached unit-spacing spectrum is rescaled per element
 * (the integrated kernel grows as h^2 on a cubic mesh, the density as h^-3).
 *   batch   : 1 .. 16 elements.
 *   sets    : device array of `batch` dks_particle_set.  An element whose
 *             x, y, z, Ex, Ey or Ez is NULL is treated as having no particles.
 *   max_np  : host bound on every element's np (at most 2^32 - 2^20); sizes the launches.
 *   scratch : device, >= dks_poisson_batch_scratch_bytes(batch, max_np),
 *             256-byte aligned, caller-owned; element b uses the b-th of
 *             `batch` equal parts (rounded down to 256 bytes).
 * Elements share nothing but the plan's read-only state, so batches on
 * different streams may run concurrently with distinct scratch buffers. */
dks_status dks_poisson_solve_particles_batched(dks_poisson_plan_t plan, int batch,
                                               const dks_particle_set* sets, int64_t max_np,
                                               void* scratch, size_t scratch_bytes,
                                               dks_stream_t stream);

/* Bytes of the library's own binned-particle scratch used by
 * dks_poisson_solve_particles_noalloc (64 MiB per GPU). */
#define DKS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* dks_poisson_solve_particles for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, hosts that forbid
 * allocation after start-up): the same step, arguments, results and errors,
 * but the binned-particle scratch is not the plan's attached one.  It is a
 * static device array of DKS_NOALLOC_SCRATCH_BYTES inside the library, one per
 * GPU, held from the first such call on that GPU until the process ends.
 * The call allocates nothing; the plan's workspace (set beforehand) is used as
 * by dks_poisson_solve_particles.
 *   np : at most the count whose dks_poisson_particle_scratch_bytes is
 *        <= DKS_NOALLOC_SCRATCH_BYTES (about 4.1 million FP32 particles, 2.3
 *        million FP64); larger counts return DKS_EWORKSPACE before any
 *        device work.
 * Every call on one GPU shares that GPU's array, through all plans: calls
 * whose device work overlaps (concurrent streams, or host threads) race and
 * give wrong results; calls ordered on one stream, or separated by a
 * synchronisation, are safe.  Nothing in the array needs clearing between
 * calls (each call writes what it reads). */
dks_status dks_poisson_solve_particles_noalloc(dks_poisson_plan_t plan, const void* x, const void* y,
                                               const void* z, int64_t np, double q, void* Ex,
                                               void* Ey, void* Ez, void* phi, int64_t* n_outside,
                                               dks_stream_t stream);

/* Charge deposit alone (CIC assignment, the "NGP, CIC, TSI" box of the OPAL
 * structure figure), including the mesh fit of a fitted plan.
 *   rho       : device [nz][ny][nx], written with the charge density, C/m^3.
 *   n_outside : device int64 counter, written; may be NULL. */
dks_status dks_poisson_deposit(dks_poisson_plan_t plan, const void* x, const void* y,
                               const void* z, int64_t np, double q, void* rho,
                               int64_t* n_outside, dks_stream_t stream);

/* Field interpolation alone (CIC gather) from a mesh field, using the
 * plan's current geometry (the explicit mesh, or the last fit).
 *   E_mesh     : device [3][nz][ny][nx], V/m, read only.
 *   Ex, Ey, Ez : device [np], written. */
dks_status dks_poisson_gather(dks_poisson_plan_t plan, const void* E_mesh, const void* x,
                              const void* y, const void* z, int64_t np, void* Ex, void* Ey,
                              void* Ez, dks_stream_t stream);

/* Read back the geometry of the last solve (or the explicit mesh):
 * h[3] cell sizes and origin[3] in metres, FP64.  Synchronises `stream`. */
dks_status dks_poisson_geometry(dks_poisson_plan_t plan, dks_stream_t stream, double* h,
                                double* origin);

/* Kernel timing (instrumentation of the library itself, not a step of the
 * method).  While enabled, every kernel a solve, deposit, gather or prepare
 * launches is bracketed by two HIP events recorded on the stream it runs on.
 * Enabling or disabling discards the records.  Not for use inside HIP graph
 * capture.  Library-wide; protected by a mutex. */
typedef struct {
  char name[40];       /* kernel name, NUL-terminated */
  int64_t launches;    /* launches recorded since timing was enabled */
  double total_ms;     /* summed event-to-event time */
  double min_ms;
  double max_ms;
} dks_kernel_time;

dks_status dks_timing_enable(int enable);

/* Wait for the recorded events, aggregate them per kernel name into
 * out[0 .. *count) (host memory, capacity entries), and drop the records.
 * DKS_EINVAL if capacity is too small (then *count is the number needed). */
dks_status dks_timing_read(dks_kernel_time* out, int capacity, int* count);

/* Host-resident offload (the paper's sequence diagram of the FFT Poisson
 * solver: the density is sent from the host, the potential comes back, and
 * streams overlap transfers with kernels).  rho comes from host memory and
 * phi / E go back to host memory.  Two device copies of the input and of the
 * outputs (the staging area) let solve k+1's upload and solve k-1's download
 * run on their own copy streams while solve k computes on the caller's
 * stream.
 *
 * Bytes of device staging area a plan needs for host-resident solves: ten
 * meshes of nx*ny*nz reals, each rounded up to a multiple of 256 bytes (two
 * slots of rho, phi and the 3-component field).  Alignment required: 256
 * bytes. */
dks_status dks_poisson_host_staging_bytes(dks_poisson_plan_t plan, size_t* bytes);

/* Attach the caller-owned device staging area (at least
 * dks_poisson_host_staging_bytes, 256-byte aligned).  Waits for every
 * host-resident solve issued on the plan to finish first.  The plan keeps the
 * pointer; the caller keeps it alive until the plan is destroyed or another
 * area is attached. */
dks_status dks_poisson_set_host_staging(dks_poisson_plan_t plan, void* staging, size_t bytes);

/* Enqueue one host-resident solve of an explicit-h plan (DKS_ESTATE on a
 * fitted plan or before prepare; DKS_EWORKSPACE without a staging area).
 *   rho_host : host [nz][ny][nx] C/m^3, read by the upload stream.
 *   phi_host : host [nz][ny][nx] volts, written by the download; may be NULL.
 *   E_host   : host [3][nz][ny][nx] V/m, written by the download; may be NULL.
 *   stream   : the compute stream of the solve's kernels.
 *   ticket   : receives the solve's sequence number (host memory).
 * At least one of phi_host, E_host must be non-NULL.  Returns without waiting
 * for any device work.  The host buffers must stay untouched until the
 * ticket is done (dks_poisson_host_query / dks_poisson_host_wait).  Overlap
 * requires page-locked host memory (hipHostMalloc); pageable memory gives the
 * same result with serialised copies.  The library owns two non-blocking copy
 * streams per plan, created on the first call on the current device; results
 * land in issue order. */
dks_status dks_poisson_solve_rho_host(dks_poisson_plan_t plan, const void* rho_host, void* phi_host,
                                      void* E_host, dks_stream_t stream, uint64_t* ticket);

/* Non-blocking: *done = 1 when the solve `ticket` has written its host
 * outputs, else 0.  DKS_EINVAL for a ticket not yet issued. */
dks_status dks_poisson_host_query(dks_poisson_plan_t plan, uint64_t ticket, int* done);

/* Block the calling thread until the solve `ticket` has written its host
 * outputs.  DKS_EINVAL for a ticket not yet issued. */
dks_status dks_poisson_host_wait(dks_poisson_plan_t plan, uint64_t ticket);

/* Release the plan's host state (the free step of section "DKS"'s usage
 * example, for the library's own part: the caller frees the buffers it
 * allocated).  Waits for outstanding host-resident solves and releases the
 * plan's copy streams.  Does not touch the caller's workspace.  NULL is
 * DKS_EINVAL; the handle is invalid afterwards. */
dks_status dks_poisson_destroy(dks_poisson_plan_t plan);

/* Static, NUL-terminated description of a status code (the error side of
 * the status-returning calls of section "DKS"'s usage example); never NULL,
 * "unknown status" for a value outside dks_status. */
const char* dks_status_string(dks_status status);

#ifdef __cplusplus
}
#endif

#endif /* DKS_POISSON_H */
