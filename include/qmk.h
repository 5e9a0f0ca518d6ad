/*
 * qmk.h -- C ABI of the MI355X AO -> MO value/gradient/Laplacian library.
 *
 * The calls follow the problem statement of the QMCkl paper (arXiv
 * 2512.16677): create a context, set the nuclei, the basis set and the MO
 * coefficients, set the electron (or grid) coordinates, get the molecular
 * orbitals with their gradients and Laplacians, destroy the context
 * (Section 5.1 usage example; Section 2.2 context and get/provide/compute
 * call structure; Section 2.3 plain C ABI with simple types).
 *
 * Conventions shared by every entry point:
 *   - Every function returns a qmk_status; 0 (QMK_OK) is success.  Functions
 *     never abort or exit.  On error the outputs are untouched, the context
 *     stays valid and qmk_last_error() returns a message.  An invalid
 *     argument returns QMK_INVALID_ARG_BASE + k, k the 1-based position of
 *     the offending argument.
 *   - Lengths are in bohr (atomic units).  Arrays are C-contiguous.
 *   - set_* calls copy their inputs: the caller may free its arrays on
 *     return.  They are synchronous.
 *   - get_* and adjoint calls write into DEVICE buffers owned by the caller
 *     (for example a torch tensor's data pointer) on the given HIP stream
 *     (NULL = the null stream); they return once the work is enqueued.  The
 *     library never frees caller memory.  Every buffer a kernel reads or
 *     writes must be accessible from the context's GPU: its device memory,
 *     managed memory, or pinned host memory mapped for the device.  Other
 *     pointers (pageable host memory) are rejected with
 *     QMK_INVALID_ARG_BASE + k before any work is enqueued.
 *   - A context is not thread-safe: use one context per host thread, as in
 *     the paper's parallelisation model (Section 2.4).  Contexts are
 *     independent of each other (Section 2.2).
 *   - Component order of every *_vgl quantity: value, d/dx, d/dy, d/dz,
 *     Laplacian (Section 3.2, equations for phi, grad phi, Laplacian phi).
 *     AOs of a shell are ordered lexicographically with the x power
 *     descending (d: xx xy xz yy yz zz; f: xxx xxy xxz xyy xyz xzz yyy yyz
 *     yzz zzz), shells in input order.
 */
#ifndef QMK_H
#define QMK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qmk_status;
typedef struct qmk_ctx_s* qmk_ctx;
typedef struct qmk_batch_s* qmk_batch;

enum {
  QMK_OK = 0,
  QMK_INVALID_CONTEXT = 1, /* NULL or destroyed context                      */
  QMK_NOT_SET = 2,         /* a prerequisite (nuclei, basis, ...) is missing */
  QMK_SIZE = 3,            /* size_max smaller than the result               */
  QMK_OUT_OF_MEMORY = 4,   /* device or host allocation failed              */
  QMK_HIP_ERROR = 5,       /* HIP runtime error; text in qmk_last_error     */
  QMK_NONFINITE = 6,       /* NaN or Inf in an input array                   */
  QMK_UNSUPPORTED = 7,     /* valid request this build does not support      */
  QMK_INVALID_ARG_BASE = 100
};

/* Precision modes (qmk_set_precision). */
enum {
  QMK_FP64 = 0,         /* FP64 AOs, FP64 MFMA contraction                   */
  QMK_MIXED_F32 = 1,    /* FP32 AOs, FP32 MFMA contraction                   */
  QMK_MIXED_BF16X3 = 2  /* FP32 AOs, three-product BF16-split MFMA contraction
                           with FP32 accumulation and compensated summation */
};

/* Element types of caller buffers. */
enum { QMK_F64 = 0, QMK_F32 = 1 };

/* Status code -> static string ("QMK_OK", ...). Never NULL.  Errors cross
 * the boundary as plain integer codes and C strings, the simple portable
 * types of the C ABI (Section 2.3, cross-language interface). */
const char* qmk_status_string(qmk_status status);

/* Last error message of a context ("" if none); valid until the next call on
 * the context.  qmk_last_error(NULL) returns the last error of a failed
 * qmk_ctx_create on this thread.  A plain C string, as every value crossing
 * the C ABI (Section 2.3); the message lives in the context, which holds
 * all per-calculation state (Section 2.2). */
const char* qmk_last_error(qmk_ctx ctx);

/* Create a context bound to HIP device `hip_device` (Section 2.2: one
 * context holds all inputs, cached intermediates and their time stamps).
 * *out receives the handle. */
qmk_status qmk_ctx_create(qmk_ctx* out, int32_t hip_device);

/* Free everything the context owns (Section 5.1, context_destroy).  The
 * handle is invalid afterwards.  Waits for the context's pending work. */
qmk_status qmk_ctx_destroy(qmk_ctx ctx);

/* Precision parameter B, bits requested (Section 3.1: default 53).  A
 * primitive of exponent g at squared distance u contributes iff
 * g*u < (B-1)*ln 2; otherwise it and all its derivatives are zero.
 * bits in 2..53.  mode: QMK_FP64, QMK_MIXED_F32 or QMK_MIXED_BF16X3; the
 * mixed modes are meant for bits = 24.  Invalidates cached results. */
qmk_status qmk_set_precision(qmk_ctx ctx, int32_t bits, int32_t mode);

/* Nuclear coordinates coord[nucl_num][3] (host memory).  nucl_num >= 1.
 * The nuclei are the centres R_A of the AOs (Section 3.1, radial and angular
 * parts), part of the wave function data a context is filled with before
 * points are set (Section 5.1, usage example).  Invalidates cached results.
 * The number of nuclei may only change while no basis is set. */
qmk_status qmk_set_nucleus(qmk_ctx ctx, int64_t nucl_num, const double* coord);

/* Contracted Cartesian Gaussian basis (Section 3.1, radial part with p = 2,
 * n_s = 0; angular part up to l = 3).  Host arrays:
 *   shell_nucleus[shell_num]       nucleus index of each shell (0-based)
 *   shell_ang_mom[shell_num]       l in 0..3
 *   shell_prim_offset[shell_num+1] primitives of shell s are
 *                                  offset[s] .. offset[s+1]-1; offset[0] = 0,
 *                                  non-decreasing, offset[shell_num] = prim_num
 *   exponent[prim_num]             gamma > 0
 *   coefficient[prim_num]          contraction coefficient a
 *   prim_factor[prim_num]          f_k, or NULL: normalised axis primitive
 *   shell_factor[shell_num]        N_s, or NULL: unit-norm contracted shell
 *   ao_factor[ao_num]              M_n, or NULL: every Cartesian AO unit-norm
 * Primitives need not be sorted: the library sorts each shell by ascending
 * exponent (Section 3.1), which makes the cutoff an early exit.  Requires
 * the nuclei.  Invalidates cached results. */
qmk_status qmk_set_basis(qmk_ctx ctx, int64_t shell_num, int64_t prim_num,
                         const int64_t* shell_nucleus, const int32_t* shell_ang_mom,
                         const int64_t* shell_prim_offset, const double* exponent,
                         const double* coefficient, const double* prim_factor,
                         const double* shell_factor, const double* ao_factor);

/* MO coefficients coef[mo_num][ao_num] (host), MO n = sum_k C[n][k] chi_k
 * (Section 3.2).  ao_num must match the basis.  Invalidates cached MOs. */
qmk_status qmk_set_mo_coef(qmk_ctx ctx, int64_t mo_num, int64_t ao_num, const double* coef);

/* Electron / grid coordinates for walk_num walkers of elec_num electrons
 * (Section 5.1, set_point).  transp = 'N': coord[walk][elec][3];
 * transp = 'T': coord[3][walk*elec].  coord_on_device = 0: host memory,
 * copied now; = 1: device memory, NOT copied -- it must hold the
 * coordinates until the last get/adjoint call that uses them has run on its
 * stream.  Increments the context's time stamp (Section 2.2), so the next
 * get recomputes every intermediate that depends on the points.
 * coord must hold 3 * walk_num * elec_num values: the library cannot check
 * the length of a plain pointer.  Errors (the context keeps its previous
 * points): QMK_INVALID_ARG_BASE + 2 (transp), + 3 (walk_num < 1, or more than
 * 2^31 points), + 4 (elec_num < 1), + 5 (NULL, or a device pointer this
 * device cannot access), + 6 (coord_on_device not 0 or 1); QMK_NONFINITE
 * for a non-finite host coordinate. */
qmk_status qmk_set_point(qmk_ctx ctx, char transp, int64_t walk_num, int64_t elec_num,
                         const double* coord, int32_t coord_on_device);

/* Dimensions; any pointer may be NULL.  point_num = walk_num * elec_num.
 * The caller sizes its result buffers from these, as the usage example of
 * Section 5.1 reads the number of MOs before evaluating them (its
 * get_mo_basis_mo_num call). */
qmk_status qmk_get_dims(qmk_ctx ctx, int64_t* nucl_num, int64_t* ao_num, int64_t* mo_num,
                        int64_t* walk_num, int64_t* elec_num);

/* AO values, gradients, Laplacians into out[walk][elec][5][ao] (device
 * buffer of size_max elements of type dtype, QMK_F64 or QMK_F32):
 * chi_n = M_n R(r) P(r) with its gradient and Laplacian with respect to the
 * electron coordinates (Section 3.1, AO, radial-part, cutoff and
 * angular-part equations).  Intended for inspection and tests: the
 * contraction consumes the AOs in the library's own layout. */
qmk_status qmk_get_ao_vgl(qmk_ctx ctx, void* out, int64_t size_max, int32_t dtype,
                          void* hip_stream);

/* MO values, gradients, Laplacians: mo_vgl[walk][elec][5][mo] =
 * sum_k C[mo][k] ao_vgl[walk][elec][5][k] (Section 3.2), into a device
 * buffer of size_max >= walk*elec*5*mo elements of type dtype.  The AO stage
 * is recomputed only if the points, basis or precision changed since it was
 * last computed (time stamps, Section 2.2). */
qmk_status qmk_get_mo_vgl(qmk_ctx ctx, void* out, int64_t size_max, int32_t dtype,
                          void* hip_stream);

/* qmk_get_mo_vgl without any allocation in the call, for callers that
 * cannot allocate device or host memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  Same arguments,
 * same result as qmk_get_mo_vgl up to rounding (the product's tile comes
 * from earlier tuning decisions or the least-padded-work rule, never from
 * timing).  The AO array is placed in a 64 MiB device array of the library
 * (one per GPU, held from the first call on that GPU until the process
 * ends) instead of the context's own buffer, so one call covers at most
 * Kp * 5 * Pp * s <= 64 MiB, with Kp = ao_num rounded up to a multiple of
 * 128, Pp = walk_num * elec_num rounded up to a multiple of 256 and s = 8
 * (QMK_FP64 mode) or 4 (mixed modes); larger calls return QMK_SIZE.
 * Requires the device copies of the basis tables and MO coefficients for
 * the current precision mode, which the first qmk_get_mo_vgl after the last
 * set_nucleus / set_basis / set_mo_coef / set_precision builds: without
 * them QMK_NOT_SET.  Always the dense product (the screening switch is not
 * used; the screened product gives the same values); with the cusp
 * correction on, QMK_UNSUPPORTED.  Kernel timing does not cover this call.
 * Every call on a GPU shares that GPU's array: calls that overlap in time
 * on one GPU (other streams, other host threads) race and give wrong
 * results.  The padding of the array is cleared on every call. */
qmk_status qmk_get_mo_vgl_noalloc(qmk_ctx ctx, void* out, int64_t size_max, int32_t dtype,
                                  void* hip_stream);

/* MO values only (the value rows of Section 3.2's product; the orbital
 * evaluation on grids of Section 5.4): mo_value[walk][elec][mo] =
 * sum_k C[mo][k] chi_k(r), into a device buffer of size_max >=
 * walk*elec*mo elements of type dtype (QMK_F64 or QMK_F32).  If the full AO
 * array is current for these points its value plane is read; otherwise a
 * value-only AO kernel runs (no derivatives).  Precision follows the mode:
 * FP64, or FP32 MFMA in both mixed modes (the value product has no BF16x3
 * form). */
qmk_status qmk_get_mo_value(qmk_ctx ctx, void* out, int64_t size_max, int32_t dtype,
                            void* hip_stream);

/* Electron density of a determinant at every point (Section 5.4, density of a
 * Kohn-Sham determinant as a sum of squared MOs):
 *   rho[walk][elec] = sum_n occ[n] * phi_n(r)^2
 * occ: host array of mo_num finite occupation numbers (for a closed-shell
 * determinant, 2 for each occupied MO and 0 otherwise); MOs with occ = 0 are
 * left out of the product.  rho: device FP64 buffer of size_max >=
 * walk*elec entries, overwritten.  The squares and the occupation-weighted
 * sum are taken in the epilogue of the MO product (MO values are never
 * stored); per-tile partial sums are added in a fixed order, so the result
 * is deterministic.  Precision as for qmk_get_mo_value; partial sums are
 * FP64.  Errors: QMK_INVALID_ARG_BASE + k (NULL, occ_num != mo_num), QMK_NONFINITE
 * (an occupation is not finite), QMK_SIZE. */
qmk_status qmk_get_density(qmk_ctx ctx, const double* occ, int64_t occ_num, double* rho,
                           int64_t size_max, void* hip_stream);

/* MO cusp correction (Section 3.3).  Inside the sphere of radius r_cusp[A]
 * around nucleus A every MO is replaced by
 *   phi_i - phi_i^{s_A} + sum_{k=0..3} f_{k,i,A} |r - R_A|^k
 * (phi_i^{s_A}: the part of MO i carried by the s-type AOs on A).  The four
 * f_k per (MO, nucleus) make the value and the first and second radial
 * derivatives continuous at r_cusp[A] and satisfy the electron-nucleus cusp
 * condition (1/phi) dphi/dr = -charge[A] at the nucleus (spherical average);
 * they are computed in FP64 when first needed after the nuclei, basis,
 * precision, MO coefficients or these arrays change.
 *   charge  host [nucl_num]: nuclear charges Z_A (finite, >= 0)
 *   r_cusp  host [nucl_num]: radii (finite, >= 0; 0 = no correction at A),
 *           or NULL to switch the correction off
 * The spheres must not overlap (r_A + r_B < |R_A - R_B|).  While the
 * correction is on, qmk_get_mo_vgl applies it; qmk_get_mo_value,
 * qmk_get_density, qmk_mo_vgl_adjoint and batches return QMK_UNSUPPORTED.
 * At a point exactly on a nucleus with a sphere the corrected gradient and
 * Laplacian are not finite (the cusp). */
qmk_status qmk_set_mo_cusp(qmk_ctx ctx, int64_t nucl_num, const double* charge,
                           const double* r_cusp);

/* Screened contraction (Section 3.2: the sparsity of the AOs lowers the
 * cost of the MO product).  With enable = 1, qmk_get_mo_vgl sorts the points
 * by nearest nucleus, evaluates the AOs in that order while recording which
 * (64-point block, 16-AO chunk) pairs hold a non-zero AO, and runs an MFMA
 * product that skips, per output tile, every K stage whose AOs are zero for
 * all of the tile's points; rows are written back in the caller's order.
 * Only exact zeros (AOs beyond the exponent cutoff) are skipped, so the
 * result equals the dense product's bit for bit (up to the sign of a zero).
 * Every precision mode (FP64, FP32 and BF16x3 products).  At most 16384 AOs
 * and 16384 nuclei (QMK_UNSUPPORTED above).  qmk_mo_vgl_adjoint screens too: W is
 * reordered once into the sorted point order, G-bar tiles whose AOs are zero
 * at all of their points are stored as zeros, and dC skips point stages with
 * no non-zero AO in its columns; electron gradients equal the dense path bit
 * for bit, dL/dC and nuclear gradients agree to rounding (sums over points in
 * sorted order; the sort is stable, so runs repeat bitwise).  AO values, MO
 * values and the density keep the dense path.  enable = 0 restores the
 * default. */
qmk_status qmk_set_screening(qmk_ctx ctx, int32_t enable);

/* Fraction of (64-point block, 16-AO chunk) pairs with a non-zero AO in the
 * last screened AO evaluation (the screening density; synchronises the
 * device).  QMK_NOT_SET before the first screened evaluation. */
qmk_status qmk_get_screening_density(qmk_ctx ctx, double* active_fraction);

/* Determinant and adjugate of a batch of small matrices (Section 3.4: the
 * inverse is adj(A) / det(A); determinant and adjugate are returned
 * together because the electron gradients of a Slater determinant need
 * adj(A) without the division):
 *   a    device FP64 [batch][n][n], row-major
 *   det  device FP64 [batch]
 *   adj  device FP64 [batch][n][n], adj(A) = transpose of the cofactor matrix
 * 1 <= n <= 4: explicit cofactors (exact also for singular matrices).
 * 5 <= n <= 32: LU with partial pivoting, adj = det * A^{-1}; when the
 * factorisation meets an exactly zero pivot, det = 0 and the adjugate is
 * the rank-one cofactor matrix built from the null vectors of the
 * triangular factor (one zero pivot) or zero (two or more).  batch = 0 does nothing
 * (the pointers may then be NULL).  Runs on the context's device and the
 * given stream; uses no other context state. */
qmk_status qmk_det_adj(qmk_ctx ctx, int64_t n, int64_t batch, const double* a, double* det, double* adj,
                       void* hip_stream);

/* Three-body (electron-electron-nucleus) Jastrow factor of every walker
 * (Section 3.5), computed through the intermediate matrix
 *   P^{k,m}_{i a} = sum_{j != i} rt_ij^k Rt_ja^m,
 *   J = sum_t sum_a c[t][a] sum_i Rt_ia^((p-k+l)/2) P^{k,(p-k-l)/2}_{i a},
 * rt_ij = exp(-kappa r_ij), Rt_ia = exp(-kappa |r_i - R_a|), for the
 * context's nuclei and points (walk_num walkers of elec_num electrons; the
 * basis is not needed).  Terms t run over p = 2..nord, k = 0..p-1,
 * l = 0..p-k-2 delta(k,0), each ascending, keeping those with p-k-l even
 * (qmk_jastrow_een_terms gives the count).  The P^{k,m} with m >= 1 are one
 * MFMA product per walker and k whose epilogue applies the coefficients, so
 * P is never stored; the m = 0 terms use the nucleus-independent row sums
 * of rt^k.  c: host FP64 [n_terms][nucl_num]; j_een: device FP64
 * [walk_num], overwritten.  2 <= nord <= 8, kappa > 0.  FP64 in every
 * precision mode; deterministic.  Errors: QMK_INVALID_ARG_BASE + 2/3/4 for
 * nord, kappa, n_terms; + 5 NULL c; + 6 j_een not device memory;
 * QMK_NONFINITE for a non-finite coefficient; QMK_NOT_SET without nuclei or
 * points. */
qmk_status qmk_jastrow_een_terms(int64_t nord, int64_t* n_terms);
qmk_status qmk_jastrow_een(qmk_ctx ctx, int64_t nord, double kappa, int64_t n_terms, const double* c,
                           double* j_een, void* hip_stream);

/* Adjoint of L = sum(W * mo_vgl) for the current points (Section 3.6 and
 * Section 3.5 motivate these derivatives; the nuclei carry their shells
 * rigidly, basis parameters are fixed):
 *   w       [walk][elec][5][mo] device buffer of type w_dtype
 *   d_coef  [mo][ao]    device FP64, dL/dC          (or NULL)
 *   d_elec  [walk][elec][3] device FP64, dL/dr      (or NULL)
 *   d_nucl  [nucl][3]   device FP64, dL/dR_nucleus  (or NULL)
 * Outputs are overwritten (not accumulated).  AO derivatives up to third
 * order (for d_elec and d_nucl) are recomputed from the coordinates, never
 * stored.  d_coef needs the AO values themselves: by default the product
 * reads the AO array that the forward pass left for the same points
 * (Section 2.2: a value is kept until one of its inputs changes); see
 * qmk_set_ao_retention.  Deterministic: the same inputs give bitwise the
 * same outputs.  The context may copy w into an internal buffer with padded
 * rows (FP64 weights in the FP32 mode, rounded to FP32; weights whose rows
 * of 5 * mo values cannot be read in 16-byte pieces); w itself is only
 * read. */
qmk_status qmk_mo_vgl_adjoint(qmk_ctx ctx, const void* w, int32_t w_dtype, double* d_coef,
                              double* d_elec, double* d_nucl, void* hip_stream);

/* AO values in the adjoint (Section 2.2 keeps a computed value until its
 * inputs change; the differentiation pattern may instead evaluate the AO
 * values again in the backward pass):
 *   retain = 1 (default): the dC product of qmk_mo_vgl_adjoint reads the AO
 *            array of the last forward pass when the points are unchanged;
 *   retain = 0: qmk_mo_vgl_adjoint evaluates the AO array again (one more AO
 *            kernel launch; with screening on, the point sort and activity
 *            bitmap too).
 * The outputs are bitwise the same either way.  QMK_INVALID_ARG_BASE + 2 for
 * any other value. */
qmk_status qmk_set_ao_retention(qmk_ctx ctx, int32_t retain);

/* Number of kernel launches issued by the context so far (for tests of the
 * time-stamp logic). */
qmk_status qmk_get_launch_count(qmk_ctx ctx, int64_t* count);

/* Kernel timing (tracing).  With timing enabled, every kernel the context
 * launches is bracketed by two HIP events recorded on the launch stream;
 * qmk_get_timing waits for the recorded events and returns the summed
 * device time (ms) and the number of launches of one kernel class since
 * timing was last enabled.  qmk_set_timing(ctx, 1) also resets the sums. */
enum {
  QMK_KERNEL_AO = 0,         /* AO value/gradient/Laplacian stage      */
  QMK_KERNEL_MO = 1,         /* AO -> MO contraction                   */
  QMK_KERNEL_GBAR = 2,       /* adjoint: W C product                   */
  QMK_KERNEL_AO_ADJOINT = 3, /* adjoint: AO derivatives contracted     */
  QMK_KERNEL_DCOEF = 4,      /* adjoint: W^T ao split-K product        */
  QMK_KERNEL_REDUCE = 5,     /* deterministic reductions               */
  QMK_KERNEL_DENSITY = 6,    /* MO values squared and summed (density) */
  QMK_KERNEL_CUSP = 7,       /* MO cusp correction                     */
  QMK_KERNEL_SORT = 8,       /* point sort of the screened contraction */
  QMK_KERNEL_DET = 9,        /* determinants and adjugates             */
  QMK_KERNEL_JASTROW = 10,   /* Jastrow: rescaled distances, final sum */
  QMK_KERNEL_JASTROW_P = 11, /* Jastrow: the P product on MFMA         */
  QMK_KERNEL_CONVERT = 12,   /* adjoint: W rounded to FP32 or split into
                                bf16 hi / lo planes (mixed modes)       */
  QMK_KERNEL_CLASSES = 13
};
qmk_status qmk_set_timing(qmk_ctx ctx, int32_t enable);
qmk_status qmk_get_timing(qmk_ctx ctx, int32_t kernel_class, double* total_ms, int64_t* launches);

/* Tile shapes of the MFMA products (QMK_KERNEL_MO, QMK_KERNEL_GBAR,
 * QMK_KERNEL_DCOEF, QMK_KERNEL_DENSITY, QMK_KERNEL_JASTROW_P).  By default the library's autotuner times every tile
 * shape on the first call of each distinct product size and keeps the
 * fastest (process-wide; QMK_TUNE_CACHE=<file> persists the choices,
 * QMK_TUNE=0 picks by least padded work without timing).  qmk_set_tile
 * forces tile `tile` (0 .. count-1) for one product class of this context,
 * or restores the autotuned choice with -1; every tile gives the same
 * result up to rounding. */
qmk_status qmk_get_tile_count(qmk_ctx ctx, int32_t* count);
qmk_status qmk_set_tile(qmk_ctx ctx, int32_t kernel_class, int32_t tile);

/* ---------------------------------------------------------------------- */
/* Batches: many independent contexts -- molecules of uneven sizes, each with
 * its own walkers -- evaluated together (independent contexts: Section 2.2;
 * parallelism over them: Section 2.4).  The batch does not own the contexts
 * and reads their current inputs at every run, so set_point between runs is
 * allowed.  All contexts must be fully set (nuclei, basis, MO coefficients,
 * points), live on one device and use one precision mode.  A run whose
 * dimensions differ from the previous run re-plans (and re-times the tile
 * shapes) automatically.  Not thread-safe; contexts of a batch must not be
 * used concurrently with its runs. */
qmk_status qmk_batch_create(qmk_batch* out, const qmk_ctx* ctxs, int64_t n);
qmk_status qmk_batch_destroy(qmk_batch batch);
const char* qmk_batch_last_error(qmk_batch batch);

/* Forward mo_vgl of every context i into outs[i] (device buffer
 * [walk][elec][5][mo] of context i, element type dtype), and, if ws != NULL,
 * the adjoint of sum_i sum(ws[i] * mo_vgl_i) with weights ws[i] (device,
 * same shape and element type as outs[i]) into d_coefs[i] [mo][ao],
 * d_elecs[i] [walk][elec][3] and d_nucls[i] [nucl][3] (device FP64; any of
 * the three pointer arrays, or any entry, may be NULL to skip that output).
 * The first run of a batch shape times the tile shapes and captures the
 * stage sequence -- persistent kernels walking longest-first work lists of
 * (molecule, tile) items -- into a HIP graph on hip_stream; every run then
 * rewrites the per-molecule argument tables and launches the graph once.
 * hip_stream = NULL uses a stream of the batch and waits for completion. */
qmk_status qmk_batch_run(qmk_batch batch, void* const* outs, int32_t dtype, const void* const* ws,
                         double* const* d_coefs, double* const* d_elecs, double* const* d_nucls,
                         void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* QMK_H */
