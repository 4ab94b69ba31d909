/*
 * ndrho -- selected elements of the density matrix by nested dissection and
 * selected inversion, on one MI355X (gfx950) GPU.
 *
 * Method (T. Ozaki, "Numerically exact O(N^{7/3}) method for large-scale
 * electronic structure calculations"):
 *   rho = M0 + Im(-(4i/beta) sum_p G(alpha_p) R_p),   alpha_p = mu + i z_p/beta
 *   (Sec. II B, Eq. (8)), with G(Z) = (Z S - H)^{-1} (Eq. (6)) evaluated only
 *   on the sparsity pattern of H and S (Sec. II C): the matrix is reordered by
 *   nested dissection (Sec. II C 1), factored by block LDL^T (Eqs. (18)-(20))
 *   front by front, and selectively inverted back down the dissection tree
 *   (Eq. (21), Eqs. (38)-(39)).  M0 = S^{-1} on the pattern (the zeroth moment
 *   of G; the constant 1/2 of Eq. (7) times the spin factor 2).  The same
 *   evaluation also gives the energy density matrix (Eq. (10)), and repeated
 *   evaluations find the chemical potential (Sec. II C 3).
 *
 * Conventions for every entry point:
 *   - every call returns an int status (NDRHO_OK or a negative code); no C++
 *     exception crosses this interface;
 *   - after a non-OK status, ndrho_last_error() returns a message;
 *   - a context is not thread safe: the caller serialises calls on it;
 *   - all device work is ordered on the context's HIP stream (passes split
 *     into launch chains fork further streams from it and join them back
 *     before the pole sum);
 *   - input arrays are copied; the caller keeps ownership of all its buffers.
 *
 * CSR input format (set_structure): 0-based, n rows (1 <= n <= 2^31 - 2), row_ptr[n+1] (int64,
 * row_ptr[0] = 0, non-decreasing), col_idx[nnz] (int32, strictly increasing
 * within each row), the diagonal present in every row, the pattern
 * structurally symmetric, values H and S real symmetric on it (|a_ij - a_ji|
 * <= 1e-12 max|a|), all finite; S positive definite.
 */
#ifndef NDRHO_H
#define NDRHO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ndrho_ctx ndrho_ctx;
typedef struct ndrho_plan ndrho_plan;

enum {
  NDRHO_OK = 0,
  NDRHO_EINVAL = -1,      /* malformed argument or input matrix */
  NDRHO_ENOMEM = -2,      /* device or host allocation failed / plan exceeds memory */
  NDRHO_ENOTSPD = -3,     /* S is not positive definite (a pivot of S <= 0) */
  NDRHO_ESINGULAR = -4,   /* a zero, tiny or non-finite pivot in alpha S - H */
  NDRHO_EDEVICE = -5,     /* HIP runtime error, or no usable gfx950 device */
  NDRHO_ESTATE = -6,      /* call out of order (e.g. density_matrix before set_poles) */
  NDRHO_EUNSUPPORTED = -7 /* option not supported by the library */
};

/* Arithmetic of the front updates.  Storage, pivot-block inverses, the
 * assembly and the pole sum are FP64 (complex128) in every mode.
 *   NDRHO_FP64:       every GEMM on the FP64 matrix cores.
 *   NDRHO_MIXED_FP32: for poles away from the real axis (all but those kept
 *                     by fp64_poles, fp64_far_poles and fp64_pole_im) the
 *                     four front-update GEMMs (L = B A^{-1},
 *                     Schur update, G_UJ, G_JJ) take FP32 products with FP32
 *                     accumulation, results summed into FP64 storage.
 *   NDRHO_MIXED_BF16X3: the same GEMMs as compensated split-BF16 products:
 *                     operands rounded to FP32 are split exactly into three
 *                     bfloat16 slices and the six leading slice products run
 *                     on the BF16 matrix cores with FP32 accumulation
 *                     (accuracy of an FP32 GEMM); a launch that runs faster
 *                     with FP32 products (small fronts) takes those. */
enum { NDRHO_FP64 = 0, NDRHO_MIXED_FP32 = 1, NDRHO_MIXED_BF16X3 = 2 };

typedef struct {
  int32_t leaf_rows;    /* nested dissection stops at domains of <= leaf_rows rows (default 32) */
  int32_t precision;    /* NDRHO_FP64 (default), NDRHO_MIXED_FP32 or NDRHO_MIXED_BF16X3 */
  int32_t pole_batch;   /* poles per device pass; 0 = largest that fits the memory budget */
  double mem_fraction;  /* fraction of free device memory the workspace may use (default 0.8) */
  int32_t verbose;      /* 0 = quiet; 1: ndrho_autotune reports each timed variant on stderr */
  int32_t fp64_poles;   /* mixed mode: the fp64_poles shifts nearest the real axis stay FP64 (default 12:
                           with 12 + 12, a 40^3-site lattice with 4 orbitals and 100 poles is within
                           1e-7 of the FP64 result; smaller fronts need fewer) */
  double fp64_pole_im;  /* mixed mode: shifts with Im alpha < fp64_pole_im also stay FP64 (default 0.05) */
  int32_t fp64_far_poles; /* mixed mode: the fp64_far_poles shifts farthest from the axis stay FP64 too
                             (default 12): their residues are as large as those of the nearest ones */
  int32_t use_graph;    /* 1 (default): capture the launch sequence of an evaluation in a hipGraph and replay it */
  int32_t gemm_variant; /* mixed mode, front-update GEMMs of the low poles: -1 (default) per-launch choice
                           (heuristic, refined by ndrho_autotune); 0 FP64; 1 FP32 products on 64x64 tiles;
                           2 FP32 products on 128x128 tiles; 3 split-BF16 products on 128x128 tiles;
                           4 split-BF16 products on 64x64 tiles; 5 split-BF16 products on 128x128 tiles,
                           each element split once per stage; 6 split-BF16 products on 128x128 tiles, K by
                           16 through double-buffered bf16 planes on the 32x32x16 matrix-core shape (a
                           launch whose operands span 2^31 bytes or more runs variant 3 instead); 7 as 6
                           on sixteen waves of one 32x32 block each (same results bit for bit; the same
                           fallback).  FP32 mode accepts 0-2, split-BF16 mode 0-7 */
  int32_t fp64_small_tiles; /* FP64 GEMM launches: -1 (default) 32x32 output tiles (two waves each) where the
                               launch's problems would fill less than half of the 64x64 tiles; 0 never;
                               1 always */
  int32_t split_streams; /* mixed mode, 0-4: 0 (default) runs every pass as one launch chain, captured in
                            a hipGraph; k >= 1 runs the FP64 poles of a pass and its low-precision poles,
                            divided into k parts, as k + 1 independent launch chains on further streams
                            that the context creates (default priority), joined back before the pole sum,
                            in passes of at least 1e10 modelled flops (smaller ones run one chain); such
                            forked passes are launched directly, not captured.  The chains share the
                            compute units: on one GPU they measured no faster than one chain.  Results
                            are identical either way.  Profiling (ndrho_profile, ndrho_autotune) always
                            runs one chain */
  double long_tail;      /* screening of long-tail basis functions (Sec. II C 1, step (ii)): 0 (default)
                            off; L >= 1: in every domain of the dissection, rows whose number of
                            pattern neighbours inside the domain exceeds L times the domain's median
                            join the domain's separator before the cut is sought */
  int32_t small_fronts;  /* 0 (default): every front runs in the level launches of its depth (extend-add,
                            pivot inverse and update GEMMs as separate grouped launches).  1: the small
                            fronts (at most 64 pivot rows and 320 pivot plus update rows, with every
                            descendant small) run in fused launches instead, one per depth and direction
                            with one workgroup per (front, pole) doing the front's whole step in FP64
                            (extend-add, assembly, pivot inverse, L and the Schur update upward; the
                            G_UU gather, G_UJ and G_JJ downward).  Other values: NDRHO_EINVAL */
  int32_t pivot_variant; /* mixed mode, GEMMs of the recursive pivot-block inverse (blocks of more than 64
                            rows) for the low poles: 0 (default) FP64, as for the FP64 poles, so that the
                            pivot-block factorizations are FP64 throughout; -1 per-launch choice
                            (split-BF16 or FP32 products on 64x64 tiles where a launch's largest problem has
                            256 rows or more, else FP64; refined by ndrho_autotune); 1-7 one of the
                            gemm_variant values the precision mode accepts.  The inverses of the 64-row
                            blocks at the bottom of the recursion and the FP64 poles stay FP64 */
} ndrho_options;

/* Fill *opt with the defaults listed above. */
int ndrho_default_options(ndrho_options* opt);

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t owned
 * by the caller (the context never destroys it), or NULL for a stream owned
 * by the context.  opt: NULL for defaults.  *out receives the context.
 * Errors: EINVAL (out NULL, bad option), EDEVICE (no such device, not gfx950). */
int ndrho_create(ndrho_ctx** out, int device, void* hip_stream, const ndrho_options* opt);

/* Release every device and host resource of the context.  NULL is a no-op. */
int ndrho_destroy(ndrho_ctx* ctx);

/* Message for the last non-OK status on ctx (owned by ctx, valid until the
 * next call on ctx).  With ctx == NULL, the last error of a failed create. */
const char* ndrho_last_error(const ndrho_ctx* ctx);

/* Register one H, S pair (Sec. II, Eq. (2)): validates the CSR (format above),
 * computes the nested-dissection ordering (Sec. II C 1; geometric, from coords
 * when given as n*3 doubles of basis-function centres, row-major), the
 * front tree and index maps (the table from pattern entries to front positions,
 * Sec. II C 2), uploads
 * everything to the device, and computes M0 = S^{-1} on the pattern by one
 * real selected inversion of S, which also checks that S is positive
 * definite.  *struct_id receives the handle for later calls.
 * Host pointers only.  Errors: EINVAL (format, asymmetry, non-finite),
 * ENOTSPD (S not positive definite), ENOMEM, EDEVICE. */
int ndrho_set_structure(ndrho_ctx* ctx, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                        const double* H, const double* S, const double* coords, int32_t* struct_id);

/* As ndrho_set_structure, for a periodic system (Sec. II C 1, step (i)):
 * cell[3] holds the lengths of the periodic cell along x, y and z in the unit
 * of coords (0 = open boundary along that axis; coords required).  An overlap
 * whose coordinate difference along a periodic axis exceeds half the cell
 * length is taken to cross the cell boundary (minimum image), and the
 * dissection numbers such a neighbour by its periodic image, so that a
 * periodic lattice is cut by two-plane separators.  H and S hold the
 * couplings of the cell with its images folded onto the pattern (a Gamma-point
 * matrix); the result is the same as for any other ordering.
 * Errors: EINVAL (cell NULL or with a negative or non-finite length, coords
 * NULL), and those of ndrho_set_structure. */
int ndrho_set_structure_periodic(ndrho_ctx* ctx, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                                 const double* H, const double* S, const double* coords, const double* cell,
                                 int32_t* struct_id);

/* Replace the values of H and S of a registered structure (same pattern).
 * Recomputes M0.  Errors as set_structure. */
int ndrho_update_values(ndrho_ctx* ctx, int32_t struct_id, const double* H, const double* S);

/* Choose the poles of Eq. (8) for a structure: z_p, R_p of the continued
 * fraction of depth 2*n_poles (Eq. (7)), alpha_p = mu + i z_p/beta and
 * weights w_p = -(4/beta) R_p.  mu in the energy unit of H, beta = 1/kT in
 * its inverse.  Errors: EINVAL (n_poles < 1, beta <= 0 or non-finite). */
int ndrho_set_poles(ndrho_ctx* ctx, int32_t struct_id, double mu, double beta, int32_t n_poles);

/* General weighted sum instead of Eq. (8)'s poles: the next density_matrix
 * returns (add_m0 ? M0 : 0) + sum_k weight[k] Re G(alpha_k)_ij on the pattern,
 * with alpha_k = alpha_re[k] + i alpha_im[k] (host arrays of length n).
 * Real or near-real shifts are the caller's risk: the factorization does not
 * pivot, and a vanishing pivot returns ESINGULAR. */
int ndrho_set_shifts(ndrho_ctx* ctx, int32_t struct_id, int32_t n, const double* alpha_re,
                     const double* alpha_im, const double* weight, int32_t add_m0);

/* rho_ij on the pattern (Eq. (8), spin factor 2 included), nnz doubles in the
 * caller's CSR order.  rho_out is a host pointer (on_device = 0; the call
 * synchronises) or a device pointer on the context's device (on_device = 1;
 * the result is ready when the context stream reaches that point).
 * Errors: ESTATE (no poles set), ESINGULAR, EDEVICE, ENOMEM. */
int ndrho_density_matrix(ndrho_ctx* ctx, int32_t struct_id, double* rho_out, int32_t on_device);

/* Tr(G(alpha_k) S) = sum_ij G_ij(alpha_k) S_ji for n shifts alpha_k =
 * alpha_re[k] + i alpha_im[k] (Im alpha_k > 0, or S - H/alpha_k positive
 * definite), from the selected inversion on the pattern with FP64 front
 * updates (Sec. II C 3, Eq. (42): -(2/pi) Im Tr(G(E + i eta) S) is the density
 * of states used by the chemical-potential search).  The structure's poles are
 * not changed.  tr_re, tr_im: n values each (host).
 * Errors: EINVAL (n < 1, NULL arrays, non-finite shift), ESINGULAR, EDEVICE, ENOMEM. */
int ndrho_green_traces(ndrho_ctx* ctx, int32_t struct_id, int32_t n, const double* alpha_re, const double* alpha_im,
                       double* tr_re, double* tr_im);

/* rho as ndrho_density_matrix with on_device = 1, for callers that cannot
 * allocate device memory during the call (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the call allocates nothing.
 * Its pole workspace, pole-sum accumulator and pivot status live in a fixed
 * device array of 64 MiB (67108864 bytes) that the library holds on every
 * device it runs on until the process ends; the structure, its poles and
 * rho_out_dev (nnz doubles on the context's device, CSR order) are the
 * caller's, set up beforehand as for ndrho_density_matrix.  The poles run in
 * passes of as many as fit beside the accumulator, as one chain of plain
 * launches on the context stream (no graph, no further streams); the call
 * synchronises the stream.  The result equals ndrho_density_matrix's.
 * Every call on one device shares that device's array, which keeps the
 * contents of the last call (the call clears what it needs cleared): calls
 * that overlap on one device, from any context, race.
 * Errors: ENOMEM (one pole of the structure, with its accumulator, needs more
 * than the array holds; the message gives both sizes), EINVAL (NULL output),
 * ESTATE (no poles set), ESINGULAR, EDEVICE. */
int ndrho_density_matrix_noalloc(ndrho_ctx* ctx, int32_t struct_id, double* rho_out_dev);

/* Chemical potential with Tr(rho(mu) S) = n_ideal (the search of Sec. II C 3,
 * Eqs. (40), (44)-(46)): each step sets the structure's
 * poles at a trial mu (as ndrho_set_poles with beta, n_poles), evaluates rho
 * and its count deviation dN = Tr(rho S) - n_ideal (Eq. (40)); the trial mu
 * comes from the quadratic through the three points of smallest |dN|, both
 * signs of dN among them when available (Muller, Eqs. (45)-(46)), else the
 * line through the last two (Eq. (44), read with the denominator
 * dN_i - dN_j), else a first move of 10 kT against the sign of dN; a trial
 * outside the bracket of points with dN < 0 < dN is replaced by bisection.
 * With retarded_step = 1 and a first |dN| above one electron, the second trial
 * comes from the retarded Green function instead (Eqs. (41)-(43)):
 * -(2/pi) Im Tr(G(E + i eta) S) with eta = 0.01 eV on 2 n_poles points over
 * mu0 +- max(2 eV, 40 kT) (ndrho_green_traces, FP64), trapezoidal rule,
 * bisection on the trial mu.  It costs about as much as six FP64 density-
 * matrix evaluations of the structure and saves one or two; 0 skips it.
 * Stops when |dN| <= tol or after max_iter density-matrix evaluations.  The
 * SCF extrapolation of Eqs. (47)-(48) is not used (there is no SCF loop).
 * On return the structure's poles are set at *mu_out.
 * mu0: first trial; *mu_out: the last trial; delta_n_out (may be NULL): its
 * dN; iters_out (may be NULL): evaluations made; rho_out (host, nnz values in
 * CSR order, may be NULL): rho at *mu_out.  Not converging within max_iter
 * is not an error: check |*delta_n_out|.
 * Errors: EINVAL (mu_out NULL, n_ideal outside (0, 2n), tol <= 0,
 * max_iter < 1, bad beta or n_poles), ESINGULAR, EDEVICE, ENOMEM. */
int ndrho_find_mu(ndrho_ctx* ctx, int32_t struct_id, double n_ideal, double beta, int32_t n_poles, double mu0,
                  double tol, int32_t max_iter, int32_t retarded_step, double* mu_out, double* delta_n_out,
                  int32_t* iters_out, double* rho_out);

/* The k eigenpairs (H c = eps S c, Eq. (2)) nearest the energy xi, by the
 * block shift-invert iteration of Appendix B: B_l = X^{-1} S C_l (Eq. (B2))
 * through the factor X = L D L^T of X = alpha S - H, alpha = xi + i eta,
 * stored by one upward sweep (Eq. (B5)) and applied in the three tree passes
 * of Eqs. (B8)-(B14); then the projected problem <b|H|b> c = <b|S|b> c eps
 * (Eq. (B3)) on the real basis [Re B_l, Im B_l], with the null directions of
 * its S-metric removed, gives the next block of 16 Ritz vectors (the 16 Ritz
 * values nearest xi; the first k are the wanted ones, the rest speed the
 * iteration).  eta > 0 keeps every pivot of the unpivoted factorization
 * nonsingular (the Hermitian part of -i X is then positive definite) without
 * changing the eigenpairs, which the projection recovers from the real and
 * imaginary parts; eta = 0 factors the real X, where a tiny pivot returns
 * ESINGULAR.  The iteration stops when every wanted Ritz pair has
 * ||H c - eps S c||_2 <= tol (c S-normalised, tol in the unit of H), or
 * after max_iter iterations (not an error: check resid_out).
 * k in [1, min(16, n)].  Outputs (host): eps_out[k] ascending; c_out (may be
 * NULL) n*k, column i the eigenvector of eps_out[i] in the caller's row order,
 * c^T S c = 1 (sign arbitrary); iters_out, resid_out[k] (may be NULL).
 * Errors: EINVAL (bad k, xi, eta, tol, max_iter; eps_out NULL), ESINGULAR,
 * EDEVICE, ENOMEM. */
int ndrho_eigenstates(ndrho_ctx* ctx, int32_t struct_id, double xi, double eta, int32_t k, int32_t max_iter,
                      double tol, double* eps_out, double* c_out, int32_t* iters_out, double* resid_out);

/* Energy density matrix e on the pattern (Sec. II B, Eqs. (10)-(11)) together
 * with rho from the same selected Green functions:
 *   e = M1 + kappa M0 + sum_p Im(-(4i/beta) G(alpha_p) R_p alpha_p),
 *   kappa = (4/beta) sum_p R_p,
 * with M0 = S^-1 and M1 = S^-1 H S^-1 (the zeroth and first moments of G,
 * Eq. (12)) on the pattern.  M1 is computed on the first call for the
 * structure (and after ndrho_update_values) from G at two shifts far up the
 * imaginary axis (FP64, Richardson-extrapolated; relative error about 1e-12
 * for Hamiltonians of a few eV).  The shifts must be the poles of
 * ndrho_set_poles.  rho_out and e_out: nnz values each in the caller's CSR
 * order, host pointers (on_device = 0; the call synchronises) or device
 * pointers on the context's device (on_device = 1).  In the mixed precision
 * forms e carries the low-precision error of the mid-range poles weighted by
 * |alpha_p|, larger than rho's.
 * Errors: EINVAL (NULL output), ESTATE (no set_poles), ESINGULAR, EDEVICE, ENOMEM. */
int ndrho_energy_density_matrix(ndrho_ctx* ctx, int32_t struct_id, double* rho_out, double* e_out,
                                int32_t on_device);

/* rho and e (as ndrho_energy_density_matrix) for k distinct structures in
 * one schedule (as ndrho_density_matrix_batch); every member needs poles from
 * ndrho_set_poles, with the same n_poles and beta (mu may differ).
 * rho_outs[i], e_outs[i]: nnz values of structure struct_ids[i] each.
 * Errors: EINVAL (repeated id, mismatched poles, NULL outputs), ESTATE,
 * ESINGULAR, EDEVICE, ENOMEM. */
int ndrho_energy_density_matrix_batch(ndrho_ctx* ctx, const int32_t* struct_ids, int32_t k, double* const* rho_outs,
                                      double* const* e_outs, int32_t on_device);

/* rho for k distinct structures in one schedule: their front trees are
 * joined into one forest (planned, uploaded and given its M0 on the first
 * call for this list of ids, then cached), so every launch works on the
 * fronts of all k structures at a depth and on all poles.  The members need
 * the same shift count, weights and M0 flag (same n_poles and beta); mu, and
 * with it alpha_p, may differ per structure.  rho_outs[i] receives
 * structure struct_ids[i]'s nnz values (host or device, as on_device).
 * Errors: EINVAL (repeated id, mismatched poles), ESTATE, ESINGULAR, ENOMEM. */
int ndrho_density_matrix_batch(ndrho_ctx* ctx, const int32_t* struct_ids, int32_t k, double* const* rho_outs,
                               int32_t on_device);

/* Autotuner of the front-update GEMM launches (and, with pivot_variant = -1,
 * of the pivot-block inverse's GEMM launches) of one structure (k = 1) or of
 * a batch of k structures (as run by ndrho_density_matrix_batch): for every
 * launch it times, on one full evaluation of the current shifts per variant,
 * each gemm_variant the precision mode accepts (FP64 for all poles; FP32
 * products on 64x64 or 128x128 tiles; in split-BF16 mode also split-BF16
 * products on 128x128 tiles, on 64x64 tiles, on 128x128 tiles with one
 * split per element and stage, and on 128x128 tiles with K staged by 16 in
 * double-buffered bf16 planes; the low-precision variants apply only to the
 * poles the mode puts in low precision) and keeps the fastest.  With
 * cache_path non-NULL the choice is looked up in, or appended to, that text
 * file under a key of the plan's shape, pole count, batch size, precision and pivot_variant
 * (a line whose choice names a variant the mode does not accept is ignored).
 * FP64 mode: nothing to tune.  With opt.verbose each timed variant and the
 * choice (one digit per launch of the program) are reported on stderr.  Errors: EINVAL, ESTATE (no shifts set), EDEVICE. */
int ndrho_autotune(ndrho_ctx* ctx, const int32_t* struct_ids, int32_t k, const char* cache_path);

typedef struct {
  int64_t n, nnz;
  int32_t n_fronts, n_levels;      /* fronts of the dissection tree; depth + 1 */
  int32_t max_front_j, max_front_u;/* largest pivot block and update set */
  int32_t root_j;                  /* pivot rows of the (largest) root front */
  int32_t n_poles, pole_batch;     /* poles set; poles per device pass */
  double flops_per_pole;           /* algorithmic flop model (8 real flops per complex FMA) */
  double flops_exec_per_pole;      /* flops the kernels actually execute per pole */
  double bytes_per_pole;           /* algorithmic HBM bytes of the front data per pole */
  double factor_bytes_per_pole;    /* device bytes of the factor panels per pole */
  double workspace_bytes;          /* device workspace currently allocated */
  double last_ms;                  /* wall time of the last density_matrix (host clock) */
  int64_t launches_per_pass;       /* kernel launches of one pass over a pole batch */
  int32_t n_fp64_poles;            /* leading shifts run with FP64 front updates */
  int32_t precision;               /* the context's precision mode */
  int32_t split_passes;            /* passes of the structure's last evaluation that ran as several
                                      launch chains (split_streams) */
} ndrho_stats_t;

/* Sizes, plan model and last-call figures of one structure.  Errors: EINVAL. */
int ndrho_structure_stats(const ndrho_ctx* ctx, int32_t struct_id, ndrho_stats_t* out);

/* Figures of the context's evaluations (any argument may be NULL):
 *   ms_per_phase[4]: kernel milliseconds, since profiling was last enabled
 *     (ndrho_profile; zeros without it), of the four phases of the path:
 *     [0] assembly of alpha S - H (Sec. II C), [1] the upward block LDL^T
 *     sweep (extend-add, pivot inverses, L and Schur updates; Eqs. (18)-(20)),
 *     [2] the downward selected inversion (Eqs. (21), (38)-(39)), [3] the pole
 *     sum of Eq. (8) and its output;
 *   *flops: algorithmic flops of the last evaluation (the plan's model, 8 real
 *     flops per complex multiply-add, times the number of shifts);
 *   *hbm_bytes: algorithmic HBM bytes of the last evaluation (the plan's model
 *     of front data read and written once per pole, complex128).  Counter
 *     readings of the device's actual traffic need a profiler.
 * Errors: EINVAL (ctx NULL). */
int ndrho_stats(const ndrho_ctx* ctx, double* ms_per_phase, double* flops, double* hbm_bytes);

/* Kernel kinds reported by the profile below. */
enum { NDRHO_K_EXTADD = 0, NDRHO_K_ASSEMBLE = 1, NDRHO_K_PIVOT_INV = 2, NDRHO_K_GEMM = 3, NDRHO_K_COPY = 4,
       NDRHO_K_GATHER = 5, NDRHO_K_ACCUM = 6, NDRHO_K_GEMM_PIVOT = 7, NDRHO_K_GEMM_F32 = 8,
       NDRHO_K_GEMM_BF16X3 = 9, NDRHO_K_SMALL = 10, NDRHO_K_COUNT = 11 };
/* NDRHO_K_GEMM: FP64 front-update GEMMs; NDRHO_K_GEMM_PIVOT: FP64 GEMMs of the
 * recursive pivot-block inverse; NDRHO_K_GEMM_F32: FP32-product front updates;
 * NDRHO_K_GEMM_BF16X3: split-BF16 front updates; NDRHO_K_SMALL: the fused
 * small-front launches (small_fronts = 1). */

/* enable != 0: from now on every launch is bracketed by HIP events on the
 * context stream and its duration is added to a per-kind total (clears the
 * totals); enable == 0 stops recording.  Instrumented calls are slower. */
int ndrho_profile(ndrho_ctx* ctx, int32_t enable);
/* Per-kind totals since profiling was enabled: kernel milliseconds, useful
 * flops (complex GEMMs: 8 real flops per complex multiply-add, symmetric
 * outputs counted once), and launch counts; arrays of NDRHO_K_COUNT. */
int ndrho_profile_read(const ndrho_ctx* ctx, double* ms, double* flops, int64_t* launches);
/* Algorithmic bytes (operands read and results written once, complex128) of
 * the profiled front-update GEMM launches per kind, bytes[NDRHO_K_COUNT]
 * (zero for the other kinds).  EINVAL for NULL arguments. */
int ndrho_profile_read_bytes(const ndrho_ctx* ctx, double* bytes);
/* The same milliseconds split by dissection-tree depth of the launch:
 * ms[kind * NDRHO_PROFILE_DEPTHS + depth] (row-major, NDRHO_K_COUNT rows,
 * caller-owned, fully written); depths >= NDRHO_PROFILE_DEPTHS - 2 share the
 * second-to-last column, and launches outside the tree (pole sum, M0 set-up)
 * use the last.  EINVAL for NULL arguments. */
enum { NDRHO_PROFILE_DEPTHS = 32 };
int ndrho_profile_read_depth(const ndrho_ctx* ctx, double* ms);

/* Device memory on the context's device for callers without their own
 * allocator (e.g. a device-resident rho_out).  ndrho_device_alloc returns
 * `bytes` of device memory in *ptr (EINVAL for bytes <= 0, ENOMEM);
 * ndrho_device_free releases it (NULL is a no-op); ndrho_device_to_host
 * copies `bytes` from device `src` to host `dst` after the context stream's
 * pending work, and synchronises. */
int ndrho_device_alloc(ndrho_ctx* ctx, int64_t bytes, void** ptr);
int ndrho_device_free(ndrho_ctx* ctx, void* ptr);
int ndrho_device_to_host(ndrho_ctx* ctx, void* dst, const void* src, int64_t bytes);
/* Plain device-to-device copy kernel of `bytes` (a multiple of 16) on the
 * context stream, synchronised; also the reference for calibrating the HBM
 * byte counters of a profiler (it reads and writes exactly `bytes`). */
int ndrho_device_copy(ndrho_ctx* ctx, void* dst, const void* src, int64_t bytes);

/* ---------------- host-only utilities (no device needed) ---------------- */

/* Poles z[n_poles] (increasing) and residues R[n_poles] of the continued
 * fraction of depth 2*n_poles (Eq. (7)): f(x) = 1/2 + sum_p R_p [1/(x - i z_p)
 * + 1/(x + i z_p)].  Errors: EINVAL. */
int ndrho_cf_poles(int32_t n_poles, double* z, double* R);

/* Nested dissection and symbolic analysis only (Secs. II C 1 and II C 2), for inspection.
 * Same input rules as set_structure (values are not needed); cell as in
 * ndrho_set_structure_periodic (NULL: open boundaries); leaf_rows and
 * long_tail as in ndrho_options. */
int ndrho_plan_create(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* coords,
                      const double* cell, int32_t leaf_rows, double long_tail, ndrho_plan** out);
int ndrho_plan_destroy(ndrho_plan* plan);
const char* ndrho_plan_last_error(void);
/* Sizes: counts[0] = n_fronts, [1] = n_levels, [2] = sum |U_f|, [3] = nnz,
 * [4] = panel elements per pole (sum (J+U) J), [5] = max J, [6] = max U. */
int ndrho_plan_counts(const ndrho_plan* plan, int64_t* counts);
/* perm[k] = original index of the k-th eliminated row (n int32). Per front f
 * (postorder, children before parents): parent[f] (-1 = root), depth[f],
 * j0[f] (first permuted position of its pivot rows), nj[f], nu[f],
 * u_off[f] (offset into the concatenated update lists).  u_rows[sum U]:
 * permuted positions of every front's update rows, increasing within a front;
 * rel[sum U]: index of each update row in the parent's local (J then U) order.
 * Any pointer may be NULL to skip it. */
int ndrho_plan_export(const ndrho_plan* plan, int32_t* perm, int32_t* parent, int32_t* depth, int64_t* j0,
                      int32_t* nj, int32_t* nu, int64_t* u_off, int32_t* u_rows, int32_t* rel);
/* Per CSR entry e: out_slot[e] = offset (complex elements) of G_ij in the
 * per-pole panel storage, asm_slot[e] = offset where X_ij is assembled, or -1
 * when the transposed entry carries it; panel_off[f] = start of front f's
 * column-major (J+U) x J panel. */
int ndrho_plan_slots(const ndrho_plan* plan, int64_t* out_slot, int64_t* asm_slot, int64_t* panel_off);
/* The launch program of one pass (upward then downward; the pole sum that
 * ends a pass is not listed): per launch, its kernel kind (NDRHO_K_*), tree
 * depth, useful flops per pole and work items (tiles or descriptors).
 * *count receives the number of launches; arrays may be NULL to query it. */
int ndrho_plan_program(const ndrho_plan* plan, int64_t* count, int32_t* kind, int32_t* depth, double* flops,
                       int64_t* items);
/* Flop and byte model per pole (8 real flops per complex multiply-add). */
int ndrho_plan_model(const ndrho_plan* plan, double* flops, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* NDRHO_H */
