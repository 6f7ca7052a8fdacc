/*
 * vecchia.h -- C ABI of the MI355X (gfx950) Vecchia Gaussian-process library.
 *
 * Computes, for a Gaussian process observed at n ordered locations, the sums
 * of Algorithm 1 of James & Guinness, "Implementation and Analysis of GPU
 * Algorithms for Vecchia Approximation" (Section 3): for every observation i
 * the conditional density of y_i given its at most m nearest previously
 * ordered neighbours (the Vecchia factorisation, Section 2.1, Eq. 3) is
 * formed from the (m+1) x (m+1) covariance of the neighbourhood, Cholesky
 * factored, and its contributions to logdet, ySy, XSX, ySX, their covariance
 * parameter derivatives and the Fisher information are summed over i.  A
 * separate combine step (Section 3) turns the sums into the profile
 * log-likelihood, gradient and Fisher information, and a Fisher-scoring
 * update (Eq. 4) moves the covariance parameters.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers.  Every array argument is a DEVICE pointer owned by the caller.
 *   The library allocates no device memory, keeps no per-call state and
 *   never synchronises the stream: work is enqueued on `stream` (a
 *   hipStream_t passed as void*, NULL = the default stream) and outputs are
 *   valid once the stream has reached that point.
 * Layouts (row-major, no padding):
 *   locs[n][d]        FP64 coordinates (1 <= d <= 4; up to 32 for
 *                     VEC_FAMILY_ANISO).
 *   NNarray[n][m+1]   int32, 0-based.  Row i holds i in column 0 and its
 *                     q = min(i, m) conditioning neighbours in columns 1..q,
 *                     each a previous observation (0 <= j < i), in any order;
 *                     the remaining columns are ignored (-1 by convention).
 *   y[n], X[n][p]     FP64 response and covariates (1 <= p <= 3).
 *   covparms[P]       FP64 covariance parameters, read on the device:
 *                       VEC_FAMILY_ISO        (sigma2, rho, tau2)          P = 3
 *                       VEC_FAMILY_SPACETIME  (sigma2, rho_s, rho_t, tau2) P = 4
 *                       VEC_FAMILY_ANISO      (sigma2, rho_1..rho_d, tau2) P = d + 2
 *                     Cov(a, b) = sigma2 * (f_nu(h) + tau2 * [a == b]) with
 *                     h the range-scaled distance (space-time: the first
 *                     nspace coordinates scaled by rho_s, the rest by rho_t;
 *                     anisotropic: coordinate k scaled by rho_k),
 *                     f_0.5 = e^-h, f_1.5 = (1+h) e^-h,
 *                     f_2.5 = (1 + h + h^2/3) e^-h  (Section 4.3, Eq. 6 at
 *                     nu = 0.5; tau2 is the nugget-to-variance ratio).
 *   raw[nraw]         the sums, nraw = 2 + p*p + p + P*(2 + p*p + p) + P*P:
 *                     [logdet, ySy, XSX[p][p], ySX[p], dlogdet[P], dySy[P],
 *                      dXSX[P][p][p], dySX[P][p], ainfo[P][P]].
 *   out[nout]         nout = 1 + P + P*P + p + p*p:
 *                     [loglik, grad[P], info[P][P], betahat[p], betainfo[p][p]]
 *                     with loglik = -1/2 (n log 2pi + logdet + ySy - ySX.betahat)
 *                     (the paper's Eq. 1 is twice this), betahat = XSX^-1 ySX.
 *   status[2]         int32 on the device: status[0] = OR of VEC_FLAG_*,
 *                     status[1] = smallest observation index that raised a
 *                     flag.  vec_status_clear() resets it.
 * Errors.  Entry points return VEC_OK or a negative code.  Problems visible
 *   on the host (null pointer, unsupported size, smoothness or family,
 *   workspace too small) return VEC_EINVAL / VEC_EWORKSPACE before anything
 *   is enqueued.  Problems found on the device (non positive-definite
 *   neighbourhood covariance, malformed NNarray row, non-finite value) set
 *   flags in `status`; outputs of that call are then undefined.  Read the
 *   status after synchronising and decode it with vec_status_code().  HIP
 *   launch failures return VEC_EHIP.  Calls that share a workspace or a
 *   status word must not run concurrently on different streams.
 */
#ifndef VECCHIA_H
#define VECCHIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VEC_OK 0
#define VEC_EINVAL (-1)
#define VEC_ENOTPD (-2)
#define VEC_EBADNN (-3)
#define VEC_ENONFINITE (-4)
#define VEC_EHIP (-5)
#define VEC_EWORKSPACE (-6)

#define VEC_FLAG_NOTPD 1
#define VEC_FLAG_BADNN 2
#define VEC_FLAG_NONFINITE 4

#define VEC_FAMILY_ISO 0
#define VEC_FAMILY_SPACETIME 1
/* One range per coordinate, for the higher-dimensional inputs of Section 4
 * (Eq. 6 with rho_1..rho_d): d <= 32, m <= 63.  It runs on the kernel that
 * gives every neighbourhood a whole wave; vec_raw_sums, vec_block_sums,
 * vec_combine, vecchia_loglik_grad_info, vec_fisher_update and
 * vec_fisher_fit accept it, the other entry points return VEC_EINVAL. */
#define VEC_FAMILY_ANISO 2

typedef struct {
  int64_t n;         /* number of observations (n >= 1, n < 2^31)          */
  int32_t m;         /* neighbours per observation: NNarray has m+1 columns */
  int32_t d;         /* coordinates per location, 1..4 (ANISO: 1..32)      */
  int32_t p;         /* covariates (columns of X), 1..3                    */
  int32_t family;    /* VEC_FAMILY_ISO, _SPACETIME or _ANISO               */
  double smoothness; /* Matern smoothness nu: 0.5, 1.5 or 2.5 (fixed)      */
  int32_t nspace;    /* space-time: leading spatial coordinates, 1..d-1    */
  int32_t reserved;  /* must be 0                                          */
} vec_problem;
/* Space-time split.  With nspace = d - 1 (time the last coordinate) every
 * entry point accepts VEC_FAMILY_SPACETIME.  Any other split runs on the
 * kernel that gives each neighbourhood a whole wave, so it is accepted
 * where VEC_FAMILY_ANISO is (vec_raw_sums, vec_block_sums, vec_combine,
 * vecchia_loglik_grad_info, vec_fisher_update, vec_fisher_fit, m <= 63);
 * the other entry points return VEC_EINVAL for it. */

/* Number of covariance parameters P, raw sums, and combined outputs; a
 * negative return means the problem description is invalid. */
int vec_nparms(const vec_problem* pb);
int vec_nraw(const vec_problem* pb);
int vec_nout(const vec_problem* pb);

/* Largest m that every single-problem entry point accepts (60, the
 * neighbour count of the paper's largest setting): the loglik-only, adjoint,
 * kriging-weights and prediction passes stop there, and the batched calls at
 * m = 40.  vec_raw_sums, vec_block_sums, vecchia_loglik_grad_info and the
 * Fisher calls accept m <= 63 for every family; neighbourhoods of more than
 * 61 observations (and VEC_FAMILY_ANISO) run on a kernel that gives each
 * neighbourhood a whole wave. */
int vec_max_m(void);

/* Bytes of device workspace vec_raw_sums needs for the observation range
 * [i0, i1) on the current device (0 if the problem is invalid). */
size_t vec_workspace_bytes(const vec_problem* pb, int64_t i0, int64_t i1);

/* Sums of Algorithm 1 (Section 3) over observations i0 <= i < i1 into
 * raw[nraw] (overwritten; zeros for an empty range).  `workspace` holds at
 * least vec_workspace_bytes(pb, i0, i1) bytes of device memory, 8-byte
 * aligned, whose contents on entry do not matter.  The result is
 * deterministic for a fixed device, problem and range. */
int vec_raw_sums(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                 const double* y, const double* X, const double* covparms, int64_t i0,
                 int64_t i1, double* raw, void* workspace, size_t workspace_bytes,
                 int32_t* status, void* stream);

/* The fused per-neighbourhood kernel alone: the sums of observations
 * [i0, i1) split into *nblocks rows of partial sums, partials[*nblocks][nraw]
 * (any summation order of the rows gives the raw sums).  `partials` holds at
 * least vec_workspace_bytes(pb, i0, i1) bytes of device memory; *nblocks is
 * written on the host (0 for an empty range).  For callers that reduce
 * partial sums themselves, e.g. across devices that each own a range of
 * observations. */
int vec_block_sums(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                   const double* y, const double* X, const double* covparms, int64_t i0,
                   int64_t i1, double* partials, size_t partials_bytes, int32_t* nblocks,
                   int32_t* status, void* stream);

/* The "separate function" of Section 3: raw sums of the whole problem (all
 * n observations) to out[nout].  A singular XSX sets VEC_FLAG_NONFINITE. */
int vec_combine(const vec_problem* pb, const double* raw, double* out, int32_t* status,
                void* stream);

/* vec_raw_sums over all n observations followed by vec_combine. */
int vecchia_loglik_grad_info(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                         const double* y, const double* X, const double* covparms, double* raw,
                         double* out, void* workspace, size_t workspace_bytes, int32_t* status,
                         void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * vecchia_loglik_grad_info without the workspace argument.  The partial sums
 * go to a 2 MiB array of device memory inside the library, one per device,
 * reserved when the library's code is loaded on that device and held until
 * the process ends; its address is looked up once per device on the first
 * call.  The call allocates nothing and runs the same kernels, so raw and
 * out equal those of vecchia_loglik_grad_info bit for bit.  Problems whose
 * partial sums need more than 2 MiB (vec_workspace_bytes(pb, 0, n) > 2 MiB:
 * only families with many parameters, e.g. VEC_FAMILY_ANISO at large d)
 * return VEC_EWORKSPACE before anything is enqueued.  Every call on a device
 * shares that device's array: calls that overlap in time on one device
 * (different streams, or different host threads) race and give undefined
 * results; calls ordered on one stream are safe. */
int vecchia_loglik_grad_info_noalloc(const vec_problem* pb, const double* locs,
                                     const int32_t* NNarray, const double* y, const double* X,
                                     const double* covparms, double* raw, double* out,
                                     int32_t* status, void* stream);

/* The profile log-likelihood alone: the sums of Algorithm 1 (Section 3)
 * without the derivative and information work, then the combine step.
 * raw receives [logdet, ySy, XSX[p][p], ySX[p]] (the first 2 + p*p + p
 * entries of the raw layout; raw[nraw] is large enough), out receives
 * [loglik, betahat[p], betainfo[p][p]] (1 + p + p*p doubles).  workspace as
 * for vec_raw_sums over [0, n). */
int vec_loglik(const vec_problem* pb, const double* locs, const int32_t* NNarray, const double* y,
               const double* X, const double* covparms, double* raw, double* out, void* workspace,
               size_t workspace_bytes, int32_t* status, void* stream);

/* Reverse-mode (adjoint) gradient of the log-likelihood with respect to
 * covparms at a given mean vector betahat[p] (device), every
 * neighbourhood's factor recomputed and no derivative matrix stored.  With
 * r = y - X betahat, v the conditional variance of observation i given its
 * neighbours and z its standardised conditional residual (the last row of
 * the neighbourhood's Cholesky factor L, Algorithm 1), u = L^-T e_last and
 * alpha = Sigma_i^-1 r_i, each neighbourhood contributes
 *   d/dtheta_j [-1/2 (log v + z^2)] =
 *     -1/2 [ (u' dS_j u)(1 + z^2) - 2 z (alpha' dS_j u) ]
 * (dS_j = dSigma_i/dtheta_j, Section 3's derivative matrices).  At betahat =
 * the GLS estimate this is the gradient of the profile log-likelihood
 * (grad[] of vecchia_loglik_grad_info).
 *   grad_out   device FP64 scalar multiplying the gradient (the incoming
 *              gradient of a reverse-mode caller), or NULL for 1.
 *   loglik     device FP64 scalar receiving -1/2 (n log 2pi + logdet +
 *              r' Sigma^-1 r) at betahat under the Vecchia factorisation, or
 *              NULL.
 *   dcovparms  device FP64 [P] receiving grad_out * d loglik / d covparms.
 * workspace holds at least vec_workspace_bytes(pb, 0, n) bytes. */
int vec_loglik_adjoint(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                       const double* y, const double* X, const double* covparms,
                       const double* betahat, const double* grad_out, double* loglik,
                       double* dcovparms, void* workspace, size_t workspace_bytes,
                       int32_t* status, void* stream);

/* Kriging weights and conditional variances of observations [i0, i1): the
 * conditional density of Eq. (3) is N(b' y_s, v) with weights b of the q
 * neighbours and variance v, which the factor of Algorithm 1 gives (last row
 * of its inverse).  weights[(i - i0)][0..m-1] receives b in NNarray column
 * order (0 for the columns beyond q = min(i, m)) and weights[(i - i0)][m]
 * receives log(v / sigma2), the log conditional variance in correlation
 * units; row stride m + 1 doubles.  raw receives the sums of vec_loglik over
 * the range (its first 2 + p*p + p entries).  workspace as for
 * vec_raw_sums(pb, i0, i1). */
int vec_kriging_weights(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                        const double* y, const double* X, const double* covparms, int64_t i0,
                        int64_t i1, double* weights, double* raw, void* workspace,
                        size_t workspace_bytes, int32_t* status, void* stream);

/* Kriging prediction (the conditional Gaussian of Eq. 3 at new points): the
 * problem pb describes the observations 0..n_obs-1 followed by n - n_obs
 * prediction points appended to locs, y and X (y of a prediction point is
 * ignored; pass 0).  NN_pred holds only the prediction rows: row j (point
 * n_obs + j) is [n_obs + j, its m nearest observed points (indices <
 * n_obs)], m + 1 int32 per row; an index outside [0, n_obs), e.g. another
 * prediction point, sets VEC_FLAG_BADNN with that point's index.  With betahat the mean parameters (e.g. the
 * GLS estimate of vec_loglik):
 *   mean[j] = x_j betahat + c' Sigma_s^-1 (y_s - X_s betahat),
 *   var[j]  = Sigma_jj - c' Sigma_s^-1 c   (the observation process, nugget
 *             included; subtract sigma2 * tau2 for the latent field),
 * from the weights mode of the fused kernel.  Requires n_obs >= m.
 * workspace: vec_kriging_predict_workspace_bytes(pb, n_obs) bytes. */
size_t vec_kriging_predict_workspace_bytes(const vec_problem* pb, int64_t n_obs);
int vec_kriging_predict(const vec_problem* pb, const double* locs, const int32_t* NN_pred,
                        const double* y, const double* X, const double* covparms,
                        const double* betahat, int64_t n_obs, double* mean, double* var,
                        void* workspace, size_t workspace_bytes, int32_t* status, void* stream);

/* Nearest previously ordered neighbours on the device (the conditioning
 * sets of Section 2.1): for every observation i of the ordered points
 * locs[n][d] (1 <= d <= 32), the min(i, m) observations j < i nearest to
 * it in Euclidean distance, written as NNarray[i] = [i, nearest first, ...,
 * -1 padding] (n rows of m + 1 int32; ties in distance go to the smaller
 * index, so the result is unique).  Scale the coordinates beforehand for
 * anisotropic ranges.  m <= 64.  d <= 4: a grid search (the call reads the
 * bounding box back to the host, so it synchronises `stream` once);
 * 4 < d <= 32: an exhaustive search, O(n^2) distances (meant for the
 * higher-dimensional problems of Section 4.2, tens of thousands of points).
 * workspace: vec_ordered_nn_workspace_bytes(n, d, m) bytes. */
size_t vec_ordered_nn_workspace_bytes(int64_t n, int32_t d, int32_t m);
int vec_ordered_nn(int64_t n, int32_t d, int32_t m, const double* locs, int32_t* NNarray,
                   void* workspace, size_t workspace_bytes, void* stream);

/* Coarse-to-fine ordering of locs[n][d] (1 <= d <= 4), an approximation of
 * the maxmin ordering that Section 2.1 builds the conditioning sets on.
 * Coordinates are quantised to a 2^B grid over the bounding box,
 * B = min(max(1, ceil(log2(max(n, 2)) / d)), floor(60 / d)); the cell code
 * interleaves the grid bits (most significant first, coordinate 0 first
 * within a level) and is read bit-reversed, so coarse lattices come before
 * the finer ones between them.  Points of one cell are ranked by tie[] (any
 * finite doubles, e.g. uniform draws; equal ties by input index), and the
 * order is that of (rank in cell, reversed code, tie, index).
 * order[n] (int64) receives the input index of each position; locs_out
 * (may be NULL; must not alias locs) receives the reordered points.
 * workspace: vec_maxmin_order_workspace_bytes(n, d) bytes (0 if the
 * arguments are invalid or the device cannot be queried). */
/* Grouped Vecchia (Section 2.1: conditioning on the joint distribution of
 * several observations at once): the ordered observations 0..n-1 are split
 * into consecutive blocks, block b = [block_start[b], block_start[b + 1])
 * of 1..max_block observations, and each block's conditioning set is
 * cond[cond_start[b] .. cond_start[b + 1]), at most pb->m earlier
 * observations (each index < block_start[b]; any order).  The likelihood is
 * the product of the block conditionals p(y_B | y_N), and the raw sums are
 * those of vec_raw_sums with every term taken for the block as a whole:
 *   logdet += log det V,  ySy += e_y' V^-1 e_y, ... (V the conditional
 *   covariance of the block, e its conditional residuals),
 *   ainfo   = the expected information of the block conditionals,
 * so vec_combine and vec_fisher_update apply unchanged; blocks of one
 * observation with cond = the NNarray rows give vec_raw_sums.
 * block_start[nblocks + 1], cond_start[nblocks + 1] (int64) and
 * cond[ncond] (int32) are device arrays; pb->NNarray conventions do not
 * apply.  Limits: max_block <= 8, pb->m + max_block <= 64, d <= 4 when
 * max_block > 1, 1 + p + (P - 1) max_block <= 64.  A block that breaks
 * them, or an index out of range, sets VEC_FLAG_BADNN with the block's
 * first observation.  Where pb->m + max_block - 1 <= 60 and the family is
 * isotropic or space-time with time last, the sums run on the fused kernel
 * as one-observation conditionals (member k of a block conditioned on the
 * block's set and members 0..k-1: the same density and expected
 * information); a conditioning set longer than the observations before its
 * block is then also flagged.  workspace: vec_grouped_workspace_bytes(pb,
 * nblocks), which covers every max_block. */
size_t vec_grouped_workspace_bytes(const vec_problem* pb, int64_t nblocks);
int vec_grouped_raw_sums(const vec_problem* pb, const double* locs, const double* y,
                         const double* X, const double* covparms, int64_t nblocks,
                         const int64_t* block_start, const int64_t* cond_start,
                         const int32_t* cond, int64_t ncond, int32_t max_block, double* raw,
                         void* workspace, size_t workspace_bytes, int32_t* status, void* stream);

/* Fisher scoring (Eq. 4) on the grouped likelihood: `iters` iterations of
 * grouped sums, combine and update on covparms (device, in place); with
 * use_graph != 0 and a non-NULL stream one iteration is captured as a HIP
 * graph and replayed.  raw, out as for vec_fisher_fit. */
int vec_grouped_fisher_fit(const vec_problem* pb, const double* locs, const double* y,
                           const double* X, double* covparms, int64_t nblocks,
                           const int64_t* block_start, const int64_t* cond_start,
                           const int32_t* cond, int64_t ncond, int32_t max_block, int32_t iters,
                           double max_step, double* raw, double* out, void* workspace,
                           size_t workspace_bytes, int32_t* status, int32_t use_graph,
                           void* stream);

size_t vec_maxmin_order_workspace_bytes(int64_t n, int32_t d);
int vec_maxmin_order(int64_t n, int32_t d, const double* locs, const double* tie, int64_t* order,
                     double* locs_out, void* workspace, size_t workspace_bytes, void* stream);

/* The combine step of vec_loglik on sums assembled by the caller:
 * raw_sum = raw_a + raw_b (raw_b may be NULL; 2 + p*p + p doubles each,
 * e.g. the parts of the observations evaluated by two different paths),
 * then out = [loglik, betahat[p], betainfo[p][p]] over all n
 * observations. */
int vec_combine_loglik(const vec_problem* pb, const double* raw_a, const double* raw_b,
                       double* raw_sum, double* out, int32_t* status, void* stream);

/* The sums of vec_loglik (logdet, ySy, XSX, ySX) over the observations
 * index[0..count) (device int32, each in [0, n), any order, repeats counted
 * again) into raw (its first 2 + p*p + p entries).  An entry outside
 * [0, n) sets VEC_FLAG_BADNN with its position's value ignored.  For
 * callers that evaluate a subset exactly, e.g. the observations a
 * surrogate hands back.  workspace as for vec_raw_sums(pb, 0, count). */
int vec_loglik_sums_at(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                       const double* y, const double* X, const double* covparms,
                       const int32_t* index, int64_t count, double* raw, void* workspace,
                       size_t workspace_bytes, int32_t* status, void* stream);

/* One Fisher-scoring step, Eq. (4), on phi = log(covparms):
 * g = covparms .* grad, I = diag(covparms) info diag(covparms),
 * step = I^-1 g scaled to length max_step if longer, covparms *= exp(step).
 * Reads grad and info from out[]; updates covparms in place on the device.
 * Nothing is changed if status already holds a flag or I is not positive
 * definite (the latter sets VEC_FLAG_NONFINITE). */
int vec_fisher_update(const vec_problem* pb, const double* out, double* covparms,
                      int32_t* status, double max_step, void* stream);

/* `iters` Fisher-scoring iterations (evaluate, reduce, combine, update), all
 * on the device.  With use_graph != 0 and a non-NULL stream one iteration
 * is captured once as a HIP graph and replayed (capture needs a stream of
 * its own); otherwise the kernels are launched directly.
 * covparms is updated in place, out[] holds the last evaluation (taken at
 * the parameters before the last update). */
int vec_fisher_fit(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                   const double* y, const double* X, double* covparms, int32_t iters,
                   double max_step, double* raw, double* out, void* workspace,
                   size_t workspace_bytes, int32_t* status, int32_t use_graph, void* stream);

/* ------------------------------------------------------------------------
 * Batches of independent datasets
 * ------------------------------------------------------------------------
 * Many datasets of uneven n and m, sharing d, p and the covariance family
 * (smoothness, m and covariance parameters per dataset), are evaluated in
 * persistent launches fed by a work queue: each dataset is cut into tiles
 * of consecutive observations, datasets are grouped into size classes by
 * the neighbourhood size m + 1 <= 11, 21, 31, 41 (one kernel instantiation
 * per class, VEC_NUM_CLASSES launches at most), and the workgroups of a
 * class take tiles until its queue is empty.  Every tile owns one row of
 * partial sums and each dataset's rows are added in a fixed order, so the
 * results are deterministic and equal to evaluating the datasets one by one
 * (Algorithm 1 per dataset, Section 3).
 * Arrays are the concatenation of the datasets' arrays: locs[n_total][d],
 * y[n_total], X[n_total][p]; NNarray blocks of n rows of m + 1 int32 each,
 * with indices local to the dataset (0-based, as for a single problem).
 * Per-dataset arrays: covparms[nsets][P], raw[nsets][nraw],
 * out[nsets][nout], status[nsets][2] (one status word per dataset, the
 * observation index in it local to the dataset). */

#define VEC_NUM_CLASSES 4

typedef struct {
  int32_t nsets;    /* datasets, 1..65535                                  */
  int32_t d;        /* coordinates per location, 1..4                      */
  int32_t p;        /* covariates, 1..3                                    */
  int32_t family;   /* VEC_FAMILY_ISO or VEC_FAMILY_SPACETIME              */
  int32_t nspace;   /* space-time: leading spatial coordinates, d - 1      */
  int32_t reserved; /* must be 0                                           */
  int64_t n_total;  /* rows of the concatenated locs / y / X               */
  int64_t nn_total; /* int32 entries of the concatenated NNarray blocks    */
} vec_batch;

typedef struct {
  int64_t obs_offset; /* first row of the dataset in locs / y / X          */
  int64_t nn_offset;  /* first entry of its NNarray block                  */
  int64_t n;          /* observations, 1 <= n < 2^31                       */
  int32_t m;          /* neighbours, 0..vec_max_m()                        */
  int32_t reserved;   /* must be 0                                         */
  double smoothness;  /* 0.5, 1.5 or 2.5                                   */
} vec_dataset;

/* Per size class: observations per tile (0 = the default, 32) and
 * persistent workgroups per CU (0 = as many as are resident at once). */
typedef struct {
  int32_t tile[VEC_NUM_CLASSES];
  int32_t blocks_per_cu[VEC_NUM_CLASSES];
} vec_schedule;

/* Host-side description of a plan, filled by vec_batch_make_plan and passed
 * unchanged to the calls that use the plan. */
typedef struct {
  int32_t nsets;
  int32_t count[VEC_NUM_CLASSES];   /* datasets per class                 */
  int32_t grid[VEC_NUM_CLASSES];    /* persistent workgroups per class    */
  int32_t reserved;
  int64_t ntiles[VEC_NUM_CLASSES];  /* tiles per class                    */
  int64_t rows;                     /* partial rows (all tiles)           */
  int64_t plan_bytes;               /* device bytes the plan occupies     */
  vec_schedule sched;               /* the schedule, defaults filled in   */
} vec_batch_plan;

/* Device bytes of the plan of a batch of nsets datasets (0 if invalid). */
size_t vec_batch_plan_bytes(int32_t nsets);

/* Validate the batch and its HOST array of descriptors sets[nsets], cut the
 * datasets into tiles and write the device plan to plan_dev (device memory
 * of at least vec_batch_plan_bytes(nsets) bytes).  The copy is made on
 * `stream`, which this call synchronises; the plan depends on n, m and the
 * schedule only, so one plan serves every later evaluation.  Returns
 * VEC_EINVAL for an invalid batch, descriptor (any offset or size outside
 * n_total / nn_total) or schedule. */
int vec_batch_make_plan(const vec_batch* bt, const vec_dataset* sets, const vec_schedule* sched,
                        vec_batch_plan* plan, void* plan_dev, size_t plan_dev_bytes,
                        void* stream);

/* Device workspace bytes the batched calls need with this plan. */
size_t vec_batch_workspace_bytes(const vec_batch* bt, const vec_batch_plan* plan);

/* Raw sums of every dataset: raw[nsets][nraw] (layout of vec_raw_sums). */
int vec_batch_raw_sums(const vec_batch* bt, const vec_batch_plan* plan, const void* plan_dev,
                       const double* locs, const int32_t* NNarray, const double* y,
                       const double* X, const double* covparms, double* raw, void* workspace,
                       size_t workspace_bytes, int32_t* status, void* stream);

/* vec_batch_raw_sums followed by the combine step of every dataset:
 * out[nsets][nout] (layout of vecchia_loglik_grad_info). */
int vec_batch_loglik_grad_info(const vec_batch* bt, const vec_batch_plan* plan,
                               const void* plan_dev, const double* locs, const int32_t* NNarray,
                               const double* y, const double* X, const double* covparms,
                               double* raw, double* out, void* workspace, size_t workspace_bytes,
                               int32_t* status, void* stream);

/* `iters` Fisher-scoring iterations (Eq. 4, as vec_fisher_update) of every
 * dataset at once; covparms[nsets][P] updated in place on the device, a
 * dataset whose status holds a flag keeps its parameters.  use_graph and
 * stream as for vec_fisher_fit. */
int vec_batch_fisher_fit(const vec_batch* bt, const vec_batch_plan* plan, const void* plan_dev,
                         const double* locs, const int32_t* NNarray, const double* y,
                         const double* X, double* covparms, int32_t iters, double max_step,
                         double* raw, double* out, void* workspace, size_t workspace_bytes,
                         int32_t* status, int32_t use_graph, void* stream);

/* Reset status[nsets][2] to "no flag" (a kernel). */
int vec_batch_status_clear(int32_t* status, int32_t nsets, void* stream);

/* Reset status to "no flag" (a kernel, safe inside graph capture). */
int vec_status_clear(int32_t* status, void* stream);

/* Map a status word copied to the host to a return code (VEC_OK or the
 * most severe of VEC_EBADNN, VEC_ENOTPD, VEC_ENONFINITE). */
int vec_status_code(const int32_t* host_status);

#ifdef __cplusplus
}
#endif

#endif /* VECCHIA_H */
