/*
 * mra.h -- C ABI of libmra.so: one multi-reference-alignment (MRA) pass of
 * 2-D classification on an AMD Instinct MI355X (gfx950).
 *
 * The calls follow the problem statement of Algorithm 1 (the GPU MRA
 * pass): input a set of particle images X and a set of reference images Y;
 * output the class averages Y' and the alignment parameters of every image.
 * The similarity is the ring-weighted rotational cross-correlation of Sec. 2,
 *     c(phi) = int_{r1}^{r2} int_0^{2 pi} x(r, theta) y(r, theta + phi) |r| dtheta dr,
 * evaluated on a polar grid (re-sample to polar coordinates, Sec. 2) for
 * every integer shift in the search range and for the mirrored image, via
 * FFT(x)' x FFT(y) per ring followed by an inverse FFT over angle (Sec. 3).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Images are float32, row-major [L][L]; pixel (x = column, y = row) has
 *    its centre at integer coordinates; the sampling centre is
 *    (floor(L/2), floor(L/2)); the image is zero outside [0, L-1]^2.
 *  - Rings r = r_min..r_max carry weight w_r = r (the |r| of the integral);
 *    angles theta_j = 2 pi j / n_phi run from +x towards +y.
 *  - CC[k, s, m, a] = sum_r w_r sum_j p_{s,m}[r][j] * qhat_k[r][(j + a) mod n_phi],
 *    p_{s,m} the bilinear polar samples of the particle at centre + s
 *    (mirror m: samples taken at angle -theta_j), qhat_k the reference's
 *    samples divided by their weighted ring norm when normalize = 1.
 *  - The winner maximises CC over (k, m, s, a); on exact ties the smallest
 *    flat index  iota = (((k*M + m)*(2T+1) + (sy+T))*(2T+1) + (sx+T))*n_phi + a
 *    wins (M = 2 with mirror search, else 1).  The reported in-plane angle is
 *    psi = (n_phi - a) mod n_phi, so particle ~ Shift_s o Mirror^m o Rot(psi*2pi/n_phi)(ref).
 *
 * Memory, streams, errors
 * -----------------------
 *  - Every array pointer is a DEVICE pointer (e.g. torch tensor.data_ptr()).
 *    The caller owns inputs and outputs and keeps them alive until the work
 *    has completed; the library owns copies of loaded references and its
 *    workspace.
 *  - Calls are asynchronous on the stream given to mra_create; results are
 *    valid after the caller synchronises that stream (or an event recorded
 *    on it).  mra_load_refs is the exception: it synchronises the stream
 *    once, to check reference norms.
 *  - Every entry point returns MRA_OK (0) or a negative MRA_E_* code.  No C++
 *    exception, abort or exit crosses the ABI.  When validation fails nothing
 *    is enqueued and outputs are untouched.  After a HIP runtime error the
 *    context is failed: every later call returns MRA_E_DEVICE until
 *    mra_destroy.  mra_last_error() gives the context's last message.
 *  - A context is not thread-safe; use one context per host thread.  Several
 *    contexts may share a device and run concurrently on different streams.
 */
#ifndef MRA_H
#define MRA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MRA_OK = 0,
  MRA_E_INVAL = -1,       /* bad argument or geometry                       */
  MRA_E_NOREF = -2,       /* refset id not loaded                            */
  MRA_E_NOMEM = -3,       /* device allocation failed or exceeds the cap     */
  MRA_E_DEVICE = -4,      /* HIP runtime error; the context is now failed    */
  MRA_E_DEGENERATE = -5,  /* a reference has zero weighted ring norm         */
};

enum { MRA_FP32 = 0, MRA_BF16 = 1, MRA_FP16 = 2 };

typedef struct mra_ctx mra_ctx;

/* Polar sampling geometry of a reference set.
 *  L          box size, 8 <= L <= 160
 *  r_min/max  1 <= r_min <= r_max <= 64 (integer ring radii)
 *  n_phi      angles per ring; the kernels support 256 (the paper's
 *             workloads); other values return MRA_E_INVAL
 *  shift_max  T >= 0: shifts {-T..T}^2 are searched (T <= 8)
 *  mirror     1: search the mirrored image too, 0: do not
 *  precision  MRA_FP32: FP32 correlation contraction (FP32 matrix cores);
 *             MRA_BF16 / MRA_FP16: contraction on 16-bit matrix cores with
 *             FP32 accumulation; polar sampling, FFTs, inverse FFTs and the
 *             arg-max stay FP32, and the winner's CC is re-scored in FP32.
 *  normalize  1: divide each reference by its weighted ring norm, 0: raw CC
 *  rescore_rows  MRA_BF16 / MRA_FP16 only.  0 or 1: the FP32 re-score covers
 *             the 16-bit winner alone.  k in 2..8: the winners of each
 *             particle's k best rows (shifts) of the 16-bit pass, and their
 *             neighbours one angle step either side (3k candidates), are
 *             re-scored in FP32 and the best of them is the result, which
 *             settles most near-ties that 16-bit rounding decides wrongly.
 *             Ignored for MRA_FP32.  MRA_E_INVAL outside 0..8. */
typedef struct mra_geom {
  int32_t L, r_min, r_max, n_phi, shift_max, mirror, precision, normalize;
  int32_t rescore_rows;
} mra_geom;

/* Per-particle alignment parameters, structure of arrays of length N
 * (device pointers).  cc2 and flat_index may be NULL. */
typedef struct mra_result {
  int32_t* ref;
  int32_t* shift_x;
  int32_t* shift_y;
  int32_t* psi;
  int32_t* mirror;
  float* cc;
  float* cc2;          /* optional: best CC over every other candidate (all
                          shifts, mirrors, references and angles but the
                          winner; equal to cc on a tie), from a second
                          contraction pass with the winner left out, in the
                          form's contraction precision.  NULL skips the pass. */
  int32_t* flat_index; /* optional: iota of the winner                      */
  float* psi_frac;     /* optional: sub-step in-plane angle in psi's units
                          (steps of 2 pi / n_phi, in [0, n_phi)): a parabola
                          through the FP32 CC at the winning angle and its two
                          neighbours peaks at a + d, |d| <= 1/2 (d = 0 if the
                          three do not curve down); psi_frac = psi - d.  One
                          more pass over the images; NULL skips it.          */
} mra_result;

/* One stack of an uneven batch (mra_align_batch). */
typedef struct mra_stack {
  int32_t refset_id;
  const float* parts;  /* [N][L][L], L of the refset                        */
  int64_t N;
  int32_t shift_max;   /* < 0: the refset's shift_max                       */
  mra_result out;
} mra_stack;

/* Create a context on `device` whose work is enqueued on `hip_stream` (a
 * hipStream_t; NULL = the null stream).  `workspace_cap_bytes` bounds the
 * device workspace (0 = 32 GiB); large calls are split into chunks that fit
 * (larger chunks fill the GPU with longer correlation runs). */
int mra_create(mra_ctx** out, int device, void* hip_stream, uint64_t workspace_cap_bytes);

/* Free every refset and the workspace (synchronises the stream). */
int mra_destroy(mra_ctx* ctx);

/* Reference preparation (Algorithm 1: convert y_i to polar coordinates and
 * apply the FFT).  `refs` is float32 [K][L][L] on the device.  Samples every
 * reference on the polar grid, takes the per-ring spectra, folds in w_r,
 * 1/norm and the inverse-DFT scale and keeps them resident under
 * `refset_id` (replacing an existing one).  Errors: MRA_E_INVAL (geometry or
 * K < 1), MRA_E_DEGENERATE (zero norm with normalize = 1), MRA_E_NOMEM. */
int mra_load_refs(mra_ctx* ctx, int32_t refset_id, const float* refs, int32_t K,
                  const mra_geom* g);

/* Validate a geometry for K references searched over shifts {-T..T}^2
 * (T = shift_max, or g->shift_max when shift_max < 0) without a context or
 * a device: returns MRA_OK when mra_load_refs and mra_align would accept
 * it, else MRA_E_INVAL.  Besides the ranges above, the flat candidate index
 * is an int32, so K * M * (2T+1)^2 * n_phi must be below 2^31 (M = 2 with
 * mirror search: with mirrors at most 85 598 references at T = 3 and
 * 14 513 at T = 8; use several refsets beyond that), and
 * the box plus search range must fit the resampler's LDS staging. */
int mra_check_geom(const mra_geom* g, int32_t K, int32_t shift_max);

/* Free one refset.  MRA_E_NOREF if absent. */
int mra_unload_refs(mra_ctx* ctx, int32_t refset_id);

/* K and geometry of a loaded refset (host pointers). */
int mra_refset_info(mra_ctx* ctx, int32_t refset_id, int32_t* K, mra_geom* g);

/* Multi-reference alignment of N particles (Algorithm 1, inner loops and the
 * reduction of Fig. 2): for every particle, every shift, both mirrors and
 * every reference, the CC over all n_phi angles, then the arg-max.  `parts`
 * is float32 [N][L][L]; `out` arrays have length N.  N = 0 is a no-op.
 * A refset with one reference (K = 1) runs a fused kernel (resampling, ring
 * FFTs, correlation, inverse FFT, arg-max and cc2 in one launch, FP32 for
 * every precision, no workspace): the single-reference pass of RFA.
 * Errors: MRA_E_NOREF, MRA_E_INVAL, MRA_E_NOMEM. */
int mra_align(mra_ctx* ctx, int32_t refset_id, const float* parts, int64_t N,
              mra_result* out);

/* mra_align for callers that cannot allocate device memory during the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results as mra_align, bit for bit, but
 * the per-chunk buffers (particle operand, row results, FP16 scales, the
 * runner-up's winner copy) live in a fixed 256 MiB device array that every
 * device the library runs on holds from mra_create until the process ends,
 * instead of the context's workspace.  Nothing is allocated or freed and no
 * memset node is recorded: padding is cleared by a kernel.  The refset must
 * already be loaded (mra_load_refs allocates).  Large N is processed in
 * chunks that fit the array (about 140 particles per chunk at L = 76, 49
 * shifts, 35 rings), so throughput is lower than mra_align's with its
 * multi-GiB workspace.  All calls on one device share its array: calls that
 * overlap in time on one device (several streams, contexts or threads) race
 * and give undefined results; serialise them.  Errors: as mra_align, and
 * MRA_E_INVAL if one particle's buffers exceed the array (not reachable
 * within the geometry limits above). */
int mra_align_noalloc(mra_ctx* ctx, int32_t refset_id, const float* parts, int64_t N,
                      mra_result* out);

/* Class-average update (Algorithm 1: apply the alignment parameters to each
 * image, compute new Y' from the aligned images).  For each class k with
 * n_k > 0:  Y'_k(u) = (1/n_k) sum_{ref_n = k} Bil(X_n; c + s_n + Mir^{m_n} Rot(psi_n 2pi/n_phi)(u - c)),
 * Mir = diag(1, -1); classes with no member keep their previous image.
 * `averages` float32 [K][L][L] is in/out (in: previous Y, out: Y'); `counts`
 * int32 [K] receives n_k.  `params` may come from mra_align or the caller
 * (ref, shift_x, shift_y, psi, mirror are read).  The sum over a class runs
 * in a fixed order, so the result is deterministic. */
int mra_update_averages(mra_ctx* ctx, int32_t refset_id, const float* parts, int64_t N,
                        const mra_result* params, float* averages, int32_t* counts);

/* Iterative MRA: the outer repeat of Algorithm 1 (Sec. 2: align against
 * the current averages, assign each particle the best reference, rebuild
 * the averages, iterate).  Pass i loads `averages` as the references of
 * `refset_id` (geometry `g`, K classes; a tuning set on that id carries over
 * when its geometry and K equal these), aligns all N particles into `out`
 * and updates `averages` and `counts` as mra_update_averages does.  The
 * paper gives no convergence rule; this one stops after pass i >= 2 when at
 * most max_changed_frac * N particles changed class since pass i - 1, or
 * after max_iter passes.
 *  averages   float32 [K][L][L] device, in: initial references, out: the
 *             averages after the last pass
 *  out        the last pass's parameters (cc2, if non-NULL, costs a second
 *             contraction on every pass)
 *  counts     int32 [K] device: class sizes of the last pass
 *  n_iter     host: passes run
 *  changed    host int64 [max_iter] or NULL: changed[i-1] = particles whose
 *             class differs from pass i-1 (changed[0] = N)
 * On return the refset holds the references of the last pass (not the new
 * averages).  Synchronises the stream once per pass.  Errors: MRA_E_INVAL
 * (N < 1, max_iter < 1, max_changed_frac outside [0, 1], NULL pointers,
 * bad geometry), and those of mra_load_refs and mra_align. */
int mra_classify(mra_ctx* ctx, int32_t refset_id, const mra_geom* g, const float* parts, int64_t N,
                 float* averages, int32_t K, int32_t max_iter, double max_changed_frac,
                 mra_result* out, int32_t* counts, int32_t* n_iter, int64_t* changed);

/* Reference-free alignment (RFA; the GPU ISAC routine that Sec. 2 builds
 * the MRA on and Sec. 5 benchmarks): the iterative loop of mra_classify
 * with one running average as the only reference.  With start_from_mean = 1
 * `average` is first set to the plain mean of the N particles; otherwise it
 * is the starting reference.  Pass i aligns every particle against
 * `average` (all shifts, both mirrors if g->mirror, all angles; the
 * fused K = 1 kernel) and rebuilds it from the aligned particles.  The
 * paper gives no stop rule; this one stops after pass i >= 2 when at most
 * max_changed_frac * N particles changed any parameter (shift, angle,
 * mirror) since pass i - 1, or after max_iter passes.
 *  average  float32 [L][L] device, in/out
 *  out      the last pass's parameters (ref = 0); cc2 costs nothing extra
 *  n_iter, changed  as in mra_classify (changed[0] = N)
 * The refset id is loaded with K = 1 and geometry g on every pass.
 * Errors as mra_classify. */
int mra_rfa(mra_ctx* ctx, int32_t refset_id, const mra_geom* g, const float* parts, int64_t N,
            float* average, int32_t start_from_mean, int32_t max_iter, double max_changed_frac,
            mra_result* out, int32_t* n_iter, int64_t* changed);

/* Alignment of several stacks of uneven size (each against its own refset,
 * with its own shift range) in one call.  Stacks are cut into pieces that
 * fill the workspace; pieces with the same precision and tile variant share
 * one persistent correlation launch (workgroups pull (stack, row tile) work
 * items until all are done) and one launch of each per-particle kernel.
 * Each stack's results equal those of mra_align on it alone.  Errors as
 * mra_align, checked for every stack before anything is enqueued. */
int mra_align_batch(mra_ctx* ctx, const mra_stack* stacks, int32_t n);

/* Tile configuration of a refset's correlation kernel (chosen by the
 * autotuner in paper_2011_05755_amd/autotune.py, or left at the default).
 *  corr_variant  -1: default for the geometry.  FP32: 0 = 8 waves with the
 *                particle operand held in registers (R4 = ceil(n_rings/4) <= 9),
 *                1 = 4 waves, operand in registers (R4 <= 12), 2 = 8 waves,
 *                operand streamed (any R4).  BF16/FP16: 0 = operand converted
 *                once per row tile and held in registers, 1 = operand re-read
 *                and converted per reference tile.  MRA_E_INVAL if the variant
 *                cannot serve the geometry.
 *  chunk_particles  particles per chunk (0: derived from the workspace cap);
 *                also caps the pieces mra_align_batch cuts the refset's stacks into.
 *  prune         -1 or 1: skip the inverse FFT over angle of every (particle
 *                row, reference) pair whose upper bound on the CC (from its
 *                spectrum: exact magnitudes of the 32 lowest frequency slots,
 *                Cauchy-Schwarz over the energy of the rest) lies below the
 *                best so far of the pair's row, or of any row of the same
 *                particle, so it cannot win; 0: evaluate every pair.
 *  run_tiles     consecutive 8-row tiles one correlation workgroup takes in
 *                order, carrying each particle's best from one tile to the
 *                next (longer runs prune more, shorter ones balance the
 *                launch better); 0: chosen from the launch size (up to 8
 *                while every CU gets 3 runs, up to 48 while it gets 20),
 *                else 1..64.
 * Results do not depend on the tuning (bit for bit). */
typedef struct mra_tuning {
  int32_t corr_variant;
  int32_t chunk_particles;
  int32_t prune;
  int32_t run_tiles;
} mra_tuning;
int mra_set_tuning(mra_ctx* ctx, int32_t refset_id, const mra_tuning* t);
int mra_get_tuning(mra_ctx* ctx, int32_t refset_id, mra_tuning* t);

/* Debug exports (same kernels as the production path).
 *  mra_debug_polar:    float32 [N][S][n_rings][n_phi] unmirrored polar
 *                      samples, S = (2T+1)^2 shifts ordered (sy, sx).
 *  mra_debug_spectra:  float32 [N][S][n_rings][n_phi/2 + 1][2] ring spectra
 *                      P_f = sum_j p_j exp(-2 pi i f j / n_phi).
 *  mra_debug_cctable:  float32 [N][K][M][2T+1][2T+1][n_phi] full CC table.
 *  mra_debug_refs:     qhat float32 [K][n_rings][n_phi], norm float64 [K]. */
int mra_debug_polar(mra_ctx* ctx, int32_t refset_id, const float* parts, int64_t N, float* out);
int mra_debug_spectra(mra_ctx* ctx, int32_t refset_id, const float* parts, int64_t N, float* out);
int mra_debug_cctable(mra_ctx* ctx, int32_t refset_id, const float* parts, int64_t N, float* out);
int mra_debug_refs(mra_ctx* ctx, int32_t refset_id, float* qhat, double* norm);

/* Kernel timing for measurement.  mra_profile(ctx, 1) clears and starts
 * recording a HIP event pair around every launch of the named kernel groups
 * ("polar", "corr", "merge", "rescore", "maxabs", "averages", "corr2" for
 * the runner-up pass of cc2, "rfa" for the fused K = 1 kernel and "refine"
 * for psi_frac) on the context's stream;
 * mra_profile(ctx, 0) stops.  mra_profile_read synchronises the stream and
 * returns the summed device time and the launch count of one group. */
int mra_profile(mra_ctx* ctx, int enable);
int mra_profile_read(mra_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches);

const char* mra_last_error(mra_ctx* ctx);
const char* mra_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* MRA_H */
