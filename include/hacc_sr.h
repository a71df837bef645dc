/*
 * hacc_sr — short-range particle-particle gravity on one MI355X (gfx950).
 *
 * The operation is the short-range half of the split-force N-body method of
 * Habib et al. 2012, "The Universe at Extreme Scale: Multi-Petaflop Sky
 * Simulation on the BG/Q" (arXiv:1211.4864):
 *
 *   a_i = sum_{j != i, s_ij < r_cut^2} m_j f(s_ij) d_ij,
 *   d_ij = x_j - x_i (minimum image in a periodic box),  s_ij = d_ij . d_ij,
 *   f(s) = (s + eps)^(-3/2) - poly5(s)                 (Sec. III, Eq. 7)
 *
 * where poly5 is the fitted grid force, eps the short-distance softening,
 * and the short-range condition s < r_cut^2 is applied inside the pair
 * kernel (Sec. III, paragraph after Eq. 7).  r_cut is the matching scale of
 * the long- and short-range forces (3 grid cells, Sec. II).  The gravitational
 * constant is 1 and the force is attractive.
 *
 * Conventions shared by every entry point:
 *
 *  - Every array argument is DEVICE memory owned by the caller, except
 *    `poly`, which is a HOST array of 6 floats c_0..c_5 (poly5(s) =
 *    sum_k c_k s^k).  Positions, velocities and per-particle vectors are
 *    row-major (n, 3) arrays, as a contiguous (n, 3) tensor.
 *  - The library never allocates device memory.  Entry points that need
 *    scratch space take it from the workspace registered with
 *    hacc_sr_set_workspace (size from hacc_sr_workspace_bytes).  Calls are
 *    asynchronous on the stream registered with hacc_sr_set_stream (the
 *    null stream by default) and return before the GPU work ends.
 *  - box > 0: periodic cube [0, box)^3; positions outside are wrapped and
 *    pair separations use the minimum image.  box < 0: open boundaries over
 *    [0, -box)^3; particles outside are clamped into the edge cells, which
 *    keeps the neighbour search exact because cells are at least r_cut wide.
 *    This is the mode for an overloaded sub-volume (Sec. II, particle
 *    overloading), shifted so that its lower corner is the origin.
 *  - Particles are binned into a chaining mesh of N^3 cells, N =
 *    floor(|box| / r_cut), so every pair inside r_cut lies in adjacent
 *    cells.  Results are returned in the caller's particle order.
 *  - Arithmetic: pair terms in float32 on cell-relative coordinates shifted
 *    into a frame centred on the work item, compensated float32
 *    accumulation; float64 only for positions, velocities and the
 *    kick/stream update.  Results are bitwise reproducible run to run.
 *  - Return codes: HACC_SR_OK, or one of the negative codes below.
 *    Argument checks run on the host before any GPU work, so a call that
 *    fails validation touches no device memory.  n == 0 is a valid no-op.
 *    The library is not thread-safe: the registered stream, workspace and
 *    timing state are process-wide host state, read when a call is made.
 *    Work queued on different streams may overlap on the device, so such
 *    calls must each register their own workspace (or the caller must order
 *    the streams): two calls in flight on one workspace race.
 */
#ifndef HACC_SR_H
#define HACC_SR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HACC_SR_OK 0
#define HACC_SR_EINVAL (-1)   /* null pointer, n < 0, r_cut/eps <= 0, non-finite scalar */
#define HACC_SR_EDOMAIN (-2)  /* periodic box < 3 r_cut, n >= 2^31, too many cells,
                                 2 min(n, cells) + n/64 >= 2^31 work items */
#define HACC_SR_ENOSPACE (-3) /* workspace unset or smaller than required */
#define HACC_SR_EHIP (-4)     /* HIP runtime error; text via hacc_sr_strerror */
#define HACC_SR_ESTALE (-5)   /* hacc_sr_force_vjp_binned: the token's binning is gone */

/* Library version, major * 10000 + minor * 100 + patch. */
int hacc_sr_version(void);

/* sha256 (64 hex digits) of the sources the library was built from: the
 * names and bytes of its HIP sources and headers.  A binding compares it
 * with the sources it ships with and refuses a stale library. */
const char *hacc_sr_source_hash(void);

/* Text for a return code; for HACC_SR_EHIP, the last HIP error message. */
const char *hacc_sr_strerror(int code);

/* Register the HIP stream (a hipStream_t passed as void*) for later calls;
 * NULL selects the null stream. */
int hacc_sr_set_stream(void *stream);

/* Chaining-mesh cells per axis for (box, r_cut): N = floor(|box| / r_cut). */
int hacc_sr_grid_dim(double box, float r_cut, int32_t *cells_per_axis);

/* Workspace bytes needed by any entry point for n particles. */
int hacc_sr_workspace_bytes(int64_t n, double box, float r_cut, size_t *bytes);

/* Register caller-owned device memory as the workspace (256-byte aligned).
 * The library keeps the pointer until the next call; the caller keeps the
 * memory alive while work that uses it may still run on the stream. */
int hacc_sr_set_workspace(void *dev_ptr, size_t bytes);

/*
 * Chaining-mesh binning (the cell list of the particle-particle part of a
 * P^3M code, Sec. II).  Outputs, all caller-owned device arrays:
 *   cell_start (N^3 + 1) int32: particles of cell c are sorted entries
 *       [cell_start[c], cell_start[c+1]); cell index c = (cx * N + cy) * N + cz.
 *   perm (n) int32: sorted entry k holds input particle perm[k].  Within a
 *       cell, particles are ordered by the Morton code of their sub-cell
 *       (the cell split into S^3 equal sub-cells, S = 4 when the cell index
 *       and the code fit in 31 bits, else 2 or 1) and then by input index,
 *       so the order is deterministic.
 *   sorted_rec (n, 4) float32: (x - x_c, y - y_c, z - z_c, m) per sorted
 *       entry, the position relative to its cell's lower corner, rounded
 *       from float64 to float32.
 * Uses the workspace.
 */
int hacc_sr_bin(const double *pos, const float *mass, int64_t n, double box,
                float r_cut, int32_t *cell_start, int32_t *perm,
                float *sorted_rec);

/*
 * Short-range accelerations (Sec. III, Eq. 7 with the cut-off applied per
 * pair).  pos: (n,3) float64; mass: (n) float32; eps > 0 (length^2);
 * poly: HOST float[6]; out_acc: (n,3) float32, input order, overwritten.
 * Bins the particles (into the workspace), builds the cell work list and
 * runs the pair kernel.
 */
int hacc_sr_force(const double *pos, const float *mass, int64_t n, double box,
                  float r_cut, float eps, const float *poly, float *out_acc);

/*
 * Vector-Jacobian product of the accelerations with respect to positions:
 * for L = sum_i g_i . a_i, out_grad_pos[k] = dL/dx_k =
 *   sum_j K_kj (m_k g_j - m_j g_k),  K = f(s) I + 2 f'(s) d d^T,
 * the derivative of the pair term of Eq. 7 (Sec. III) with respect to both
 * end points; the jump of f at r_cut is ignored.  grad_acc: (n,3) float32
 * cotangents g; out_grad_pos: (n,3) float64, input order, overwritten.
 * Re-bins from pos.
 */
int hacc_sr_force_vjp(const double *pos, const float *mass, int64_t n,
                      double box, float r_cut, float eps, const float *poly,
                      const float *grad_acc, double *out_grad_pos);

/*
 * Reuse of a binning for the VJP.  hacc_sr_force and hacc_sr_force_vjp
 * leave their binning (sorted records, permutation, cell table, ordered work
 * list) in the workspace; hacc_sr_binning_token names it (0: none).  Any
 * other call that writes the workspace (binning, RCB, plain, PM, full step,
 * pair count, probe), and any change of stream or workspace, retires it;
 * kicks, streams and hacc_sr_force_noalloc do not.
 *
 * hacc_sr_force_vjp_binned is hacc_sr_force_vjp at the positions and
 * masses of the call that left the binning named by `token`, without
 * binning again: it reads them from the kept records, so later changes to
 * the position array do not matter.  n, box and r_cut must equal that
 * call's; eps and poly may differ.  Returns HACC_SR_ESTALE, before any GPU
 * work, when the token is 0, retired, or names another size or geometry;
 * the caller then uses hacc_sr_force_vjp.  In a stream-kick-stream step the
 * reverse pass's VJP at the subcycle's force position is such a call.
 */
int hacc_sr_binning_token(uint64_t *token);
int hacc_sr_force_vjp_binned(uint64_t token, int64_t n, double box, float r_cut,
                             float eps, const float *poly, const float *grad_acc,
                             double *out_grad_pos);

/*
 * RCB fat leaves (Sec. III: the short-range solver's recursive coordinate
 * bisection tree, nodes split at the centre of mass along the longest side
 * of their bounding box, particles partitioned into disjoint contiguous
 * child ranges, fat leaves sharing one interaction list).  The chaining
 * mesh stays the coarse level: inside every cell with more than leaf_max
 * particles the particles are reordered by the cell's RCB tree, cut until
 * every leaf holds at most leaf_max (1 <= leaf_max <= 2^20; else
 * HACC_SR_EINVAL).  A node whose particles all lie on one side of the
 * centre of mass (coincident particles) is cut in two by index.  Leaves
 * never cross cells.  The _rcb entry points need the workspace size from
 * hacc_sr_workspace_bytes_rcb.
 *
 * hacc_sr_rcb_bin: the binning of hacc_sr_bin followed by the leaves.
 * Outputs (caller-owned device arrays): cell_start, perm, sorted_rec as for
 * hacc_sr_bin (cell_start is the same; the order inside each cell is the
 * tree's); leaf_start (n + 1) int32: leaf l is sorted entries
 * [leaf_start[l], leaf_start[l + 1]), for l < *n_leaves (device int32).
 * nodes, node_split, n_nodes may all be NULL; otherwise nodes (n, 4) int32
 * receives every internal node as (first entry, count, count of the left
 * child, axis 0..2, or 3 for an index cut), node_split (n) float32 its
 * split coordinate (cell-relative, as in sorted_rec), *n_nodes (device
 * int32) their number, in no particular order.
 */
int hacc_sr_workspace_bytes_rcb(int64_t n, double box, float r_cut, size_t *bytes);
int hacc_sr_rcb_bin(const double *pos, const float *mass, int64_t n, double box,
                    float r_cut, int32_t leaf_max, int32_t *cell_start,
                    int32_t *perm, float *sorted_rec, int32_t *leaf_start,
                    int32_t *n_leaves, int32_t *nodes, float *node_split,
                    int32_t *n_nodes);

/*
 * hacc_sr_force and hacc_sr_force_vjp with the RCB leaves as the work
 * items: each leaf is one work item of at most 64 targets (larger leaves
 * are cut into 64-target items in tree order) whose sources are the
 * particles of the 27 cells around it within r_cut of the item's bounding
 * box, staged once and shared by all its targets.  Same arguments, outputs
 * and accuracy as the chaining-mesh entry points, plus leaf_max.  Each call
 * synchronises the stream once, to read the number of leaves.
 */
int hacc_sr_force_rcb(const double *pos, const float *mass, int64_t n, double box,
                      float r_cut, float eps, const float *poly, int32_t leaf_max,
                      float *out_acc);
int hacc_sr_force_vjp_rcb(const double *pos, const float *mass, int64_t n,
                          double box, float r_cut, float eps, const float *poly,
                          int32_t leaf_max, const float *grad_acc,
                          double *out_grad_pos);

/*
 * hacc_sr_force for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same kernels and results, with no workspace.  Its scratch memory is a
 * file-scope device array of 128 MiB in the library, which every GPU the
 * library runs on holds until the process ends; a call whose workspace
 * (hacc_sr_workspace_bytes for the same n, box, r_cut) exceeds 128 MiB
 * returns HACC_SR_ENOSPACE before any GPU work (about a million particles
 * at a few per cell).  No allocation, no event, no memset: buffers that
 * must start at zero are cleared by kernels.  Every call on one GPU uses
 * that GPU's one array, so calls that may overlap on one GPU (two streams,
 * two threads) race; the caller must order them.  Runs on the registered
 * stream; the registered workspace is neither used nor changed.
 */
int hacc_sr_force_noalloc(const double *pos, const float *mass, int64_t n,
                          double box, float r_cut, float eps, const float *poly,
                          float *out_acc);

/*
 * Plain versions of hacc_sr_force and hacc_sr_force_vjp at the same
 * accuracy, for comparison only: one thread per target, sources read from
 * global memory over the 27 stencil cells, the cut-off as a branch, the same
 * float32 pair arithmetic and sums in float64; no LDS tiling, culling or
 * work list.  Same arguments, outputs and binning as the main entry points.
 */
int hacc_sr_force_plain(const double *pos, const float *mass, int64_t n,
                        double box, float r_cut, float eps, const float *poly,
                        float *out_acc);
int hacc_sr_force_vjp_plain(const double *pos, const float *mass, int64_t n,
                            double box, float r_cut, float eps,
                            const float *poly, const float *grad_acc,
                            double *out_grad_pos);

/*
 * Long-range accelerations from the spectral particle-mesh solver (Sec. II):
 * Cloud-In-Cell deposit of the masses on a periodic grid of ng^3 cells of
 * side D = box / ng (grid point g at g D), the isotropising filter of Eq. 5
 * exp(-k^2 (sigma D)^2 / 4) [sin(k D / 2) / (k D / 2)]^n_s (sigma in grid
 * cells; nominal 0.8 and 3), the sixth-order periodic influence function
 * (read as the inverse of the sixth-order central-difference Laplacian's
 * symbol), fourth-order spectral differencing of the potential (read as the
 * fourth-order central difference's symbol), one inverse FFT per component
 * and CIC interpolation to the particles.  G = 1, a = -grad phi,
 * nabla^2 phi = 4 pi rho, the mean density removed (phi(0) = 0).
 * pos (n,3) float64, positions wrapped into [0, box); mass (n) float32;
 * box > 0 (periodic only); ng a power of two, 8..512; out_acc (n,3)
 * float32, input order, overwritten.  Float32 grids and FFTs; the deposit
 * sums in fixed point, so results are bitwise reproducible.  Uses the
 * workspace (size from hacc_sr_pm_workspace_bytes for the same ng and n:
 * two complex ng^3 grids and the buffers of a sort of the n particles by
 * grid cell); n < 2^31 - 1.
 */
int hacc_sr_pm_workspace_bytes(int32_t ng, int64_t n, size_t *bytes);
int hacc_sr_pm_accel(const double *pos, const float *mass, int64_t n, double box,
                     int32_t ng, float sigma, int32_t n_s, float *out_acc);

/*
 * One full time step of the split-operator scheme (Sec. II, Eq. 6):
 *   M_full(dt) = M_lr(dt/2) (M_sr(dt/n_c))^n_c M_lr(dt/2),
 * in place on pos and vel ((n,3) float64; pos wrapped into [0, box)).  M_lr
 * kicks the velocities with the long-range PM acceleration of
 * hacc_sr_pm_accel (positions frozen); M_sr is the stream-kick-stream
 * subcycle with the short-range force of hacc_sr_force at step dt / n_c.
 * Newtonian coefficients (v += t a, x += t v); the cosmological factors
 * are not printed in the paper.  box > 0 (periodic); the PM arguments as
 * for hacc_sr_pm_accel, the short-range ones as for hacc_sr_force; n_c >= 1.
 * acc_scratch: (n,3) float32 device array, overwritten.  Needs the larger
 * of the two workspace sizes (hacc_sr_workspace_bytes, hacc_sr_pm_workspace_bytes).
 */
int hacc_sr_full_step(double *pos, double *vel, const float *mass, int64_t n,
                      double box, int32_t ng, float sigma, int32_t n_s, float r_cut,
                      float eps, const float *poly, double dt, int32_t n_c,
                      float *acc_scratch);

/*
 * Kick of the stream-kick-stream subcycle (Sec. II, Eq. 6):
 * vel[k] += dt * acc[k] over the 3n components, in float64.
 */
int hacc_sr_kick(double *vel, const float *acc, int64_t n, double dt);

/*
 * Stream of the stream-kick-stream subcycle (Sec. II, Eq. 6):
 * pos[k] += dt * vel[k] over the 3n components, in float64, then wrapped
 * into [0, box) when box > 0 (no wrap when box <= 0).
 */
int hacc_sr_stream(double *pos, const double *vel, int64_t n, double dt,
                   double box);

/*
 * Adjoint of the kick with respect to the acceleration: grad_acc[k] =
 * float32(dt * grad_vel[k]) over the 3n components.  Used by the reverse
 * pass of a subcycle rollout.
 */
int hacc_sr_kick_adjoint(const double *grad_vel, float *grad_acc, int64_t n,
                         double dt);

/*
 * Work accounting for the pair kernel (not needed to compute forces):
 * out_counts[0] = candidate pairs (i, j != i) the kernel evaluates,
 * out_counts[1] = pairs with s < r_cut^2 (the test taken in float32 as in
 * the pair kernel).  out_counts: DEVICE int64[2], overwritten.
 */
int hacc_sr_count_pairs(const double *pos, int64_t n, double box, float r_cut,
                        float eps, int64_t *out_counts);

/*
 * Kernel timing with HIP events recorded on the library stream around each
 * launch of a pair kernel.  kernel: 0 = forward pair kernel, 1 = VJP pair
 * kernel, 2 = binning (all its kernels), 3 = work-list build, 4 = plain
 * forward kernel, 5 = plain VJP kernel, 6 = RCB tree and leaf table,
 * 7 = long-range PM solve (hacc_sr_pm_accel).
 * hacc_sr_timing_enable(1) starts recording (and clears earlier records);
 * hacc_sr_timing_read waits for the recorded events and returns the number
 * of launches and their summed duration in milliseconds.
 */
int hacc_sr_timing_enable(int enable);
int hacc_sr_timing_read(int kernel, int64_t *launches, double *total_ms);

/*
 * Rate probe of the float32 vector ALU, for measurement only: the peak the
 * pair kernels are held to, at the shader clock the chip sustains under a
 * VALU load.  kind 0: float32 fused multiply-add; 1: float32 reciprocal
 * square root; 2: one reciprocal square root per 18 multiply-adds (the
 * forward pair term's mix); 3: float32 multiply-add into its destination
 * (the short v_fmac_f32 encoding).  16 independent chains per lane,
 * waves_per_simd (1..8) one-wave workgroups per SIMD of the device, 5 timed
 * launches.  Uses the workspace (about 2.2 MB; HACC_SR_ENOSPACE if smaller)
 * and synchronises the stream.  out: HOST double[4]: [0] lane operations
 * per second (an FMA counts as one operation, 2 FLOP), [1] mean shader
 * clock during the loops in GHz, [2] shader cycles between two consecutive
 * instructions of one wave, [3] milliseconds per launch.
 */
int hacc_sr_valu_probe(int kind, int waves_per_simd, double *out);

#ifdef __cplusplus
}
#endif

#endif /* HACC_SR_H */
