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
 *    The library is not thread-safe: stream, workspace and timing state are
 *    process-wide.
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

/* Library version, major * 10000 + minor * 100 + patch. */
int hacc_sr_version(void);

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
 * Re-bins from pos (nothing is kept from a forward call).
 */
int hacc_sr_force_vjp(const double *pos, const float *mass, int64_t n,
                      double box, float r_cut, float eps, const float *poly,
                      const float *grad_acc, double *out_grad_pos);

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
 * forward kernel, 5 = plain VJP kernel.
 * hacc_sr_timing_enable(1) starts recording (and clears earlier records);
 * hacc_sr_timing_read waits for the recorded events and returns the number
 * of launches and their summed duration in milliseconds.
 */
int hacc_sr_timing_enable(int enable);
int hacc_sr_timing_read(int kernel, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* HACC_SR_H */
