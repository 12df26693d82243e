/*
 * rtcal.h -- C ABI of the MI355X (gfx950) library for the hot path of
 * gradient-based radio-environment calibration by differentiable ray tracing
 * (Hoydis et al., "Learning Radio Environments by Differentiable Ray
 * Tracing", arXiv 2311.18558).
 *
 * The computation split follows the paper's forward model: fixed specular
 * paths (found once on the host), per-path field computation giving a
 * complex coefficient a_i and delay tau_i (Sec. II-C, II-D, Eq. cfr_cont),
 * the channel frequency response over OFDM subcarriers (Sec. II-A), a loss
 * on it, and the reverse-mode adjoints back to material and antenna
 * parameters (Sec. III, Algorithm 1).
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers owned by the caller (for example
 *    torch tensors).  The library never allocates, frees or synchronises
 *    device memory except where an entry point says otherwise; work is
 *    enqueued on `stream` (a hipStream_t passed as void*, NULL = default
 *    stream) and runs asynchronously.
 *  - Complex arrays ("c64") are interleaved {float re, float im}, the
 *    layout of torch.complex64.
 *  - Gradients of a real loss L with respect to a complex z are
 *    dL/dRe(z) + j dL/dIm(z) (the torch convention).
 *  - Host-side argument checks return a negative rtc_status and set a
 *    thread-local message readable with rtc_last_error(); nothing is
 *    enqueued then.  HIP launch errors return RTC_ERR_HIP.  Device-side
 *    data (ids, offsets) is trusted: out-of-range material ids are clamped
 *    to the last material.
 *  - Results are deterministic run to run: every reduction has a fixed
 *    order and no floating-point atomics are used.
 */
#ifndef RTCAL_H
#define RTCAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTC_ABI_VERSION 9

typedef enum {
  RTC_OK = 0,
  RTC_ERR_INVALID_ARG = -1, /* NULL pointer or nonsensical scalar          */
  RTC_ERR_SHAPE = -2,       /* sizes inconsistent with each other          */
  RTC_ERR_RANGE = -3,       /* a size beyond what the kernels support      */
  RTC_ERR_WORKSPACE = -4,   /* workspace missing or smaller than required  */
  RTC_ERR_HIP = -5,         /* a HIP runtime call failed                   */
  RTC_ERR_UNSUPPORTED = -6  /* valid request this build does not implement */
} rtc_status;

/* OFDM grid and antennas.  Subcarrier n (0..n_sc-1) is at
 *   f_n = fc_hz + (n - floor(n_sc/2)) * df_hz              (Sec. II-A)
 * The Tx is a uniform linear array of n_elem isotropic elements with
 * half-wavelength spacing along the unit vector ula_axis, centred on the Tx
 * position; the Rx is one isotropic element.  zeta_tx / zeta_rx are the
 * polarisation slant angles of the polarisation model (Sec. II-B), 0 meaning
 * vertical.  Path coefficients are evaluated at the carrier (wavelength and
 * permittivity at fc); only the delay phase varies across subcarriers. */
typedef struct {
  double fc_hz;
  double df_hz;
  int32_t n_sc;
  int32_t n_elem;
  float ula_axis[3];
  float zeta_tx;
  float zeta_rx;
} rtc_radio;

/* Specular path store (device arrays).  Paths of link l are
 * link_off[l] .. link_off[l+1]-1 (CSR, non-decreasing, link_off[0] = 0,
 * link_off[n_links] = n_paths).  Interaction k (0-based) of path p lives at
 * index k*n_paths + p of every per-interaction array (interaction-major
 * structure of arrays); slots k >= depth[p] are ignored.
 *   tx_pos, rx_pos : float [n_links*3]   link end points (metres)
 *   depth          : uint8 [n_paths]     number of interactions Q <= max_depth
 *   kind           : uint8 [max_depth*n_paths] 0 = specular reflection,
 *                    1 = diffuse (Lambertian) reflection, 2 = edge
 *                    diffraction (see edge); may be NULL (all specular)
 *   px,py,pz       : float [max_depth*n_paths] interaction points s_j
 *   nx,ny,nz       : float [max_depth*n_paths] surface unit normals (either
 *                    orientation)
 *   dA             : float [max_depth*n_paths] area element of diffuse
 *                    interactions; may be NULL when kind is NULL
 *   mat            : uint16 [max_depth*n_paths] material class ids
 *   tau            : double [n_paths] path delays (seconds), total length / c
 *   edge, mat_n    : first-order edge diffraction (Sec. II-E), or NULL: a path
 *                    of depth 1 whose interaction has kind 2 is diffracted at
 *                    the point s_1 on a wedge edge; its normal must be that of
 *                    face 0 on the free-space side and its mat that of face 0.
 *                    edge = float [4*n_paths], rows (ex, ey, ez, n): the unit
 *                    edge direction e with n0 x e pointing from the edge into
 *                    face 0, and n with exterior wedge angle n pi (0 < n <= 2);
 *                    mat_n = uint16 [n_paths] the material of face n (needed
 *                    with per-id materials; per-interaction materials give
 *                    both faces the interaction's values).  Only diffraction
 *                    paths' entries are read.  kind 2 without edge, or at any
 *                    other slot, is a specular reflection.  The coefficient
 *                    is the UTD of Kouyoumjian and Pathak with Luebbers'
 *                    finite-conductivity face coefficients (Fresnel r_perp,
 *                    r_par at the rays' grazing angles), spreading
 *                    sqrt(s'/(s (s + s'))); tau is (s' + s)/c.
 */
typedef struct {
  int32_t n_links;
  int32_t n_paths;
  int32_t max_depth;
  const int64_t* link_off;
  const float* tx_pos;
  const float* rx_pos;
  const uint8_t* depth;
  const uint8_t* kind;
  const float* px;
  const float* py;
  const float* pz;
  const float* nx;
  const float* ny;
  const float* nz;
  const float* dA;
  const uint16_t* mat;
  const double* tau;
  const float* edge;
  const uint16_t* mat_n;
} rtc_paths;

/* Materials, in exactly one of two modes.
 *  per-id:  raw = float [n_mat*3], raw parameters u per material class with
 *           eps_r = 1 + exp(u0), sigma = exp(u1), S = logistic(u2)
 *           (the trainable-material parametrisation of Sec. III-C with
 *           one-dimensional embeddings and unit read-out); per_inter = NULL.
 *  per-interaction (neural materials, Sec. III-D): per_inter = float
 *           [3 * R] holding the rows eps_r, sigma, S of length R; raw = NULL.
 *           With inter_idx = NULL the rows are indexed like the
 *           per-interaction path arrays (R = max_depth*n_paths).  Otherwise
 *           inter_idx = int32 [max_depth*n_paths] maps every used slot
 *           (k < depth[p]) to its row 0 .. n_inter-1 (R = n_inter; unused
 *           slots are not read), so that only used interactions are stored
 *           and evaluated; rtc_trace_fields_adjoint then writes dLd_inter in
 *           the same compact rows.
 * n_mat <= 512.  mu_r = 1 and the XPD coefficient does not enter specular
 * reflection. */
typedef struct {
  int32_t n_mat;
  const float* raw;
  const float* per_inter;
  const int32_t* inter_idx;
  int64_t n_inter;
} rtc_materials;

/* Trainable antenna and scattering patterns and cross-polarisation
 * (optional; see rtc_trace_fields_pat).  Members may be NULL / 0:
 *  n_vmf, tx_raw: the Tx gain of Sec. III-A, a mixture of n_vmf <= 8
 *           spherical Gaussians, G(k) = 4 pi eta sum_i (w_i/a_i) e^{lam_i mu_i.k}
 *           with a_i = (2 pi/lam_i)(e^{lam_i} - e^{-lam_i}) (the factor 4 pi
 *           makes the gain integrate to 4 pi eta, Eq. atenna_normalization);
 *           tx_raw = float [1 + 5 n_vmf]: eta = logistic(r0), w = softmax of
 *           n_vmf logits, lam = exp of n_vmf values, then n_vmf mean
 *           directions as 3-vectors of any length (normalised).  The Tx
 *           pattern is sqrt(G) (cos zeta_tx, sin zeta_tx) (Eq.
 *           polarization_model) for every array element.  n_vmf = 0: isotropic.
 *  mat_raw: float [n_mat * 6], per material id: K_x = logistic(q0), the
 *           weights (w1, w2, w3) = softmax(q1, q2, q3), lam_2 = exp(q4),
 *           lam_3 = exp(q5) of the trainable scattering pattern (Sec. III-B,
 *           Eq. trainable_scattering_pattern): a Lambertian lobe and lobes
 *           about the backscatter direction -k_in and the specular
 *           direction, each normalised by Meder's hemispherical integral for
 *           an axis at the incidence angle.  At a diffuse reflection the
 *           field is |E_s| (sqrt(1 - K_x), sqrt(K_x)) with this f_s.  NULL:
 *           Lambertian and K_x = 0. */
typedef struct {
  int32_t n_vmf;
  const float* tx_raw;
  const float* mat_raw;
} rtc_patterns;

/* Library version and the last error message of the calling thread. */
int rtc_abi_version(void);
const char* rtc_last_error(void);

/* Operations that take a workspace, for rtc_workspace_size(). */
typedef enum {
  RTC_OP_CFR_LOSS = 1,
  RTC_OP_CFR_ADJOINT = 2,
  RTC_OP_TRACE_FIELDS_ADJOINT = 3,
  RTC_OP_CFR_TARGET_STATS = 4,
  RTC_OP_PAPER_LOSS = 5,
  RTC_OP_TRACE_FIELDS_ADJOINT_PAT = 6,
  RTC_OP_VALIDATE_PATHS = 7,
  RTC_OP_CFR_LOSS_ADJOINT = 8
} rtc_op;

/* Bytes of device workspace `op` needs for n_links links (CFR rows are
 * n_links * radio->n_elem) and n_paths paths.  0 on invalid input. */
size_t rtc_workspace_size(int op, const rtc_radio* radio, int32_t n_links, int32_t n_paths,
                          int32_t n_mat);

/* Device-side check of a path store (the contract of rtc_paths): counts of
 * violations per category into counts = device int64 [RTC_N_VALIDATE],
 * deterministic (no atomics).  Categories: link_off not a CSR of n_paths
 * (RTC_VAL_LINK_OFF), depth above max_depth (RTC_VAL_DEPTH), a material id
 * of a used slot (or mat_n of a diffraction path) >= n_mat, when n_mat > 0
 * (RTC_VAL_MAT), kind above 2 (RTC_VAL_KIND), tau not finite and positive
 * (RTC_VAL_TAU), a normal or edge direction not of unit length within 1 %
 * (RTC_VAL_UNIT), a non-finite point or end point (RTC_VAL_NONFINITE), a
 * negative or non-finite dA of a diffuse slot or a wedge n outside (0, 2]
 * (RTC_VAL_RANGE).  ws: rtc_workspace_size(RTC_OP_VALIDATE_PATHS, ...)
 * bytes.  The field kernels clamp material ids and read no entry outside the
 * arrays, so an invalid store yields wrong values, not faults; this names
 * what is wrong (the Python binding runs it on every upload when the
 * environment sets RTCAL_DEBUG=1). */
enum {
  RTC_VAL_LINK_OFF = 0,
  RTC_VAL_DEPTH = 1,
  RTC_VAL_MAT = 2,
  RTC_VAL_KIND = 3,
  RTC_VAL_TAU = 4,
  RTC_VAL_UNIT = 5,
  RTC_VAL_NONFINITE = 6,
  RTC_VAL_RANGE = 7,
  RTC_N_VALIDATE = 8
};
rtc_status rtc_validate_paths(const rtc_paths* paths, int32_t n_mat, int64_t* counts, void* ws,
                              size_t ws_bytes, void* stream);

/* Per-path field computation (Sec. II-C transfer chain, Sec. II-D-1
 * specular reflection with the Fresnel coefficients of Eqs. fresnel-1/-2,
 * Eq. cfr_cont):
 *   a[p]   (c64 [n_paths])  = lambda/(4 pi) * C_R^H T_p(C_T) / (c tau_p),
 *                             the delay phase factored out
 *   psi[p] (float [n_paths]) = pi * k1_p . ula_axis, the phase step between
 *                             adjacent Tx elements for the departure
 *                             direction k1_p.
 * Either output pointer may be NULL. */
rtc_status rtc_trace_fields(const rtc_radio* radio, const rtc_paths* paths,
                            const rtc_materials* mats, void* a, float* psi, void* stream);

/* rtc_trace_fields with trainable patterns (rtc_patterns; NULL gives
 * rtc_trace_fields). */
rtc_status rtc_trace_fields_pat(const rtc_radio* radio, const rtc_paths* paths,
                                const rtc_materials* mats, const rtc_patterns* pats, void* a,
                                float* psi, void* stream);

/* Channel frequency response (Eq. cfr_cont, discrete form of Sec. II-A):
 *   H[l, m, n] = sum_{i in link l} a_i g_m exp(j psi_i (m - (M-1)/2))
 *                                  exp(-j 2 pi f_n tau_i)
 * a: c64 [n_paths], psi: float [n_paths], g: c64 [n_elem] element gains,
 * H: c64 [n_links, n_elem, n_sc] (fully overwritten).  Accuracy: the sum
 * runs on the FP16 matrix cores as two-part splits (~2^-22 relative error
 * per product, FP32 accumulation) under an exact power-of-two scale per
 * link, so any finite FP32 a and g work; measured per-link relative error
 * against an FP64 direct sum ~3e-7. */
rtc_status rtc_cfr(const rtc_radio* radio, const rtc_paths* paths, const void* a,
                   const float* psi, const void* g, void* H, void* stream);

/* Target energies of a batch of CFR rows (n_rows = n_links * n_elem rows of
 * n_sc subcarriers): stats[0] = sum |H*|^2, stats[1] = sum (p*)^2 with p* the
 * power delay profile p_l = |h[l]|^2 of the centred 1/sqrt(N) IDFT
 * (Sec. II-A).  stats: device double [2].  p_tgt: NULL, or device float
 * [n_rows * n_sc] that receives p* per row in storage order,
 * p_tgt[row, k] = |X_k|^2 / N with X_k = sum_n H*[n] exp(+j 2 pi n k / N)
 * (the centred taps up to their order), for later rtc_cfr_loss calls on the
 * same targets.  n_sc must be a power of two, 2 <= n_sc <= 4096. */
rtc_status rtc_cfr_target_stats(const rtc_radio* radio, int32_t n_links, const void* H_tgt,
                                double* stats, float* p_tgt, void* ws, size_t ws_bytes,
                                void* stream);

/* The targets in the delay domain, for rtc_cfr_loss_adjoint_cir: per row
 * (n_rows = n_links * n_elem) the unnormalised transform
 *   X_tgt[row, k] = X*_k = sum_n H*[n] exp(+j 2 pi n k / N),  k = 0..N-1
 * (c64, natural order; the same transform whose |X*_k|^2 / N is the target
 * PDP of rtc_cfr_target_stats, Sec. II-A), and the same stats (device
 * double [2]: sum |H*|^2, sum (p*)^2).  Computed once per target set, like
 * p_tgt.  X_tgt: device c64 [n_links, n_elem, n_sc], must not alias H_tgt.
 * ws: rtc_workspace_size(RTC_OP_CFR_TARGET_STATS, ...) bytes.  n_sc a power
 * of two, 2 <= n_sc <= 4096. */
rtc_status rtc_cfr_target_cir(const rtc_radio* radio, int32_t n_links, const void* H_tgt,
                              double* stats, void* X_tgt, void* ws, size_t ws_bytes,
                              void* stream);

/* Coherent + power-delay-profile loss over a batch (workload loss):
 *   L = w_coh * sum|H - H*|^2 / sum|H*|^2 + w_pdp * sum (p - p*)^2 / sum (p*)^2
 * H, H_tgt: c64 [n_links, n_elem, n_sc].  tgt_stats: device double [2] from
 * rtc_cfr_target_stats for the same H_tgt, or NULL to compute it here.
 * p_tgt: the target PDP written by rtc_cfr_target_stats for the same H_tgt
 * (saves one transform per row), or NULL to derive it from H_tgt.
 * loss: device double [3] = {L, coherent term, PDP term} (unweighted terms).
 * dLdH: c64 like H or NULL; it may alias H (in-place).  n_sc must be a power
 * of two, 2 <= n_sc <= 4096. */
rtc_status rtc_cfr_loss(const rtc_radio* radio, int32_t n_links, const void* H,
                        const void* H_tgt, const double* tgt_stats, const float* p_tgt,
                        float w_coh, float w_pdp, double* loss, void* dLdH, void* ws,
                        size_t ws_bytes, void* stream);

/* rtc_cfr_loss with the targets given as their transforms X* (X_tgt, c64
 * [n_links, n_elem, n_sc], from rtc_cfr_target_cir): the same loss and
 * dL/dH (by Parseval sum |H - H*|^2 = sum |X - X*|^2 / N, p* = |X*|^2 / N,
 * dL/dH = IDFT(2 w_coh / (N Z0) (X - X*) + 4 w_pdp / (N Z1) (p - p*) X) with
 * the unnormalised inverse), in two transforms per row instead of three.
 * tgt_stats: from rtc_cfr_target_cir, required with dLdH (without it the
 * loss is normalised by the batch's own target sums).  dLdH may alias H.
 * ws: rtc_workspace_size(RTC_OP_CFR_LOSS, ...) bytes.  n_sc a power of two,
 * 2 <= n_sc <= 4096. */
rtc_status rtc_cfr_loss_cir(const rtc_radio* radio, int32_t n_links, const void* H,
                            const void* X_tgt, const double* tgt_stats, float w_coh, float w_pdp,
                            double* loss, void* dLdH, void* ws, size_t ws_bytes, void* stream);

/* rtc_cfr_loss for callers that cannot allocate memory (code recorded into
 * a HIP graph, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments and results without the workspace.  Its workspace is a
 * fixed device array inside the library, one copy per GPU (about 16.3 MiB,
 * held until the process ends); its address on a GPU is looked up on the
 * first call there.  It calls no hipMalloc/hipFree.
 * Limit: n_links * n_elem <= rtc_cfr_loss_noalloc_max_rows() (524,288 CFR
 * rows); larger batches return RTC_ERR_RANGE with a message.  Every call on
 * one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (other streams, other host threads) race and must be serialised by the
 * caller.  Nothing in the array needs to start at zero (every value is
 * written before it is read). */
rtc_status rtc_cfr_loss_noalloc(const rtc_radio* radio, int32_t n_links, const void* H,
                                const void* H_tgt, const double* tgt_stats, const float* p_tgt,
                                float w_coh, float w_pdp, double* loss, void* dLdH,
                                void* stream);
int64_t rtc_cfr_loss_noalloc_max_rows(void);

/* CIR statistics of the paper's loss (Sec. III-E, Eqs. delay_spread and
 * channel_gain), one per row (link l, element m) of H, c64
 * [n_links, n_elem, n_sc].  The row's CIR is the centred 1/sqrt(N) IDFT of
 * Sec. II-A with taps l = -N/2 .. N/2-1 (a path of delay tau lands at
 * l = tau W, W = n_sc * df_hz); p_l = |h[l]|^2,
 *   P       = sum_l p_l                                   (total gain)
 *   tau_RMS = sqrt(sum_l (l - tbar)^2 p_l / P) / W        (seconds)
 * with tbar = sum_l l p_l / P.  A row with P = 0 gets tau_RMS = 0.
 * stats: device double [n_links * n_elem][2] = {P, tau_RMS}.  n_sc must be
 * a power of two, 2 <= n_sc <= 4096.  No workspace. */
rtc_status rtc_cir_stats(const rtc_radio* radio, int32_t n_links, const void* H, double* stats,
                         void* stream);

/* The paper's calibration loss (Sec. III-E, Eqs. loss and smape) averaged
 * over the batch as in Algorithm 1, every CIR row being one example:
 *   L = (1/B) sum_b [ w_tau l(tau_b, tau^_b) + w_gain l(alpha P_b, P^_b) ]
 * with B = n_links * n_elem, l(x, y) = |x - y| / (x + y) (0 when x + y = 0),
 * (P_b, tau_b) = tgt_stats (rtc_cir_stats of the measured CFRs) and
 * (P^_b, tau^_b) the statistics of H.
 * alpha: device double [2] = {alpha, number of updates so far}, the scale of
 *   the measurements (Sec. III-F).  With update_alpha != 0 it is first
 *   advanced by one step of Eq. scaling_param: alpha^ = sum_b P_b P^_b /
 *   sum_b P_b^2 over this batch (Eq. alpha_hat; P^_b = sum_n |H_n|^2), then
 *   alpha = alpha^ on the first update (alpha_0 = alpha^_1) and
 *   delta * alpha + (1 - delta) * alpha^ afterwards, delta in [0, 1]; if
 *   sum_b P_b^2 = 0 alpha is left unchanged.  With update_alpha = 0 the
 *   stored alpha is used as it is ({1, 0}: unscaled measurements).
 *   alpha is a constant of the gradient (estimated, not learned).
 * loss: device double [3] = {L, mean l of tau, mean l of gain}.
 * pred_stats: device double [B][2] = {P^_b, tau^_b}, or NULL.
 * dLdH: c64 like H, or NULL; it may alias H (in place).  Where l has its
 *   kink (x = y) its derivative is taken as 0, and a row whose delay
 *   profile has zero variance gets no delay-spread gradient.
 * ws: rtc_workspace_size(RTC_OP_PAPER_LOSS, ...) bytes.  n_sc as for
 *   rtc_cir_stats. */
rtc_status rtc_paper_loss(const rtc_radio* radio, int32_t n_links, const void* H,
                          const double* tgt_stats, double* alpha, int32_t update_alpha,
                          double delta, float w_tau, float w_gain, double* loss,
                          double* pred_stats, void* dLdH, void* ws, size_t ws_bytes,
                          void* stream);

/* Evaluation metrics of Sec. IV-C per measurement point (link): with the
 * gains and delay spreads of its n_elem rows averaged,
 *   ALE = |10 log10(scale * Pbar) - 10 log10(Pbar^)|     (dB)
 *   RAE = |taubar - taubar^| / taubar
 * meas, pred: device double [n_links * n_elem][2] = {P, tau_RMS} (from
 * rtc_cir_stats); scale: device double (for example alpha[0] of
 * rtc_paper_loss) or NULL for 1.  out: device double [n_links][2] =
 * {ALE, RAE}.  Zero averages give inf or NaN as IEEE arithmetic does. */
rtc_status rtc_eval_ale_rae(int32_t n_links, int32_t n_elem, const double* meas,
                            const double* pred, const double* scale, double* out, void* stream);

/* Adjoint of rtc_cfr:
 *   G[m, i]  = sum_n dLdH[l(i), m, n] exp(+j 2 pi f_n tau_i)
 *   dLda[i]  = sum_m G[m, i] conj(g_m exp(j psi_i (m - c)))      c64 [n_paths]
 *   dLdg[m]  = sum_i G[m, i] conj(a_i exp(j psi_i (m - c)))      c64 [n_elem]
 * with c = (M-1)/2.  dLdg is reduced over all links in FP64 in a fixed
 * order.  Either output may be NULL; the workspace
 * (rtc_workspace_size(RTC_OP_CFR_ADJOINT, ...)) is always required.
 * Accuracy as rtc_cfr: FP16 two-part splits, dL/dH under a power-of-two
 * scale that follows the largest value read, for any finite FP32 input. */
rtc_status rtc_cfr_adjoint(const rtc_radio* radio, const rtc_paths* paths, const void* a,
                           const float* psi, const void* g, const void* dLdH, void* dLda,
                           void* dLdg, void* ws, size_t ws_bytes, void* stream);

/* rtc_cfr, rtc_cfr_loss and rtc_cfr_adjoint as one pass per link, with H
 * and dL/dH kept on chip (never written to memory):
 *   H     = the CFR of rtc_cfr (Eq. cfr_cont at the subcarriers of
 *           Sec. II-A), FP16 two-part splits as there
 *   loss  = the workload loss of rtc_cfr_loss, device double [3] =
 *           {L, coherent term, PDP term}
 *   dLda, dLdg = rtc_cfr_adjoint applied to dL/dH of that loss (either may
 *           be NULL); dLdg reduced over the links in FP64, fixed order.
 * The targets' statistics come precomputed: tgt_stats (device double [2])
 * and p_tgt (target PDP, float [n_links * n_elem * n_sc]) from
 * rtc_cfr_target_stats of the same H_tgt (c64 [n_links, n_elem, n_sc]).
 * Shapes: 1 <= n_elem <= 32 and n_sc of 256, 512 or 1024 (a link's whole
 * CFR, 32 x 1024 subcarriers, fits one workgroup's registers); others return
 * RTC_ERR_UNSUPPORTED (use the three separate calls).  dL/dH enters the
 * adjoint under one power-of-two scale per link (its largest value below
 * 2^14), exact both ways.
 * ws: rtc_workspace_size(RTC_OP_CFR_LOSS_ADJOINT, radio, n_links, ...)
 * bytes. */
rtc_status rtc_cfr_loss_adjoint(const rtc_radio* radio, const rtc_paths* paths, const void* a,
                                const float* psi, const void* g, const void* H_tgt,
                                const double* tgt_stats, const float* p_tgt, float w_coh,
                                float w_pdp, double* loss, void* dLda, void* dLdg, void* ws,
                                size_t ws_bytes, void* stream);

/* rtc_cfr_loss_adjoint with the targets given in the delay domain: X_tgt
 * and tgt_stats from rtc_cfr_target_cir of the same H_tgt.  The loss and
 * its gradient are the same functions of H: by Parseval
 * sum_n |H - H*|^2 = sum_k |X - X*|^2 / N with X the row's transform, the
 * PDP target is |X*|^2 / N, and dL/dH = IDFT(2 w_coh / (N Z0) (X - X*) +
 * 4 w_pdp / (N Z1) (p - p*) X) with the inverse transform unnormalised.  A
 * row then reads its 8 bytes of target per subcarrier once, after its first
 * transform, instead of H* (8 bytes) and p* (4 bytes) around both.  Shapes,
 * accuracy and workspace as rtc_cfr_loss_adjoint
 * (RTC_OP_CFR_LOSS_ADJOINT). */
rtc_status rtc_cfr_loss_adjoint_cir(const rtc_radio* radio, const rtc_paths* paths,
                                    const void* a, const float* psi, const void* g,
                                    const void* X_tgt, const double* tgt_stats, float w_coh,
                                    float w_pdp, double* loss, void* dLda, void* dLdg, void* ws,
                                    size_t ws_bytes, void* stream);

/* Adjoint of rtc_trace_fields: from dLda (c64 [n_paths]) to
 *   per-id mode:          dLd_raw  float [n_mat*3], gradient w.r.t. the raw
 *                         parameters u (overwritten, FP64-accumulated)
 *   per-interaction mode: dLd_inter float [3 * R], rows dL/d eps_r,
 *                         dL/d sigma, dL/d S per interaction in the rows of
 *                         rtc_materials.per_inter (without inter_idx, slots
 *                         beyond a path's depth are set to 0)
 * The unused output must be NULL. */
rtc_status rtc_trace_fields_adjoint(const rtc_radio* radio, const rtc_paths* paths,
                                    const rtc_materials* mats, const void* dLda,
                                    float* dLd_raw, float* dLd_inter, void* ws, size_t ws_bytes,
                                    void* stream);

/* Adjoint of rtc_trace_fields_pat: as rtc_trace_fields_adjoint, plus
 *   dLd_tx  float [1 + 5 n_vmf] gradient w.r.t. tx_raw, or NULL
 *           (needs n_vmf > 0; either material mode)
 *   dLd_pat float [n_mat * 6] gradient w.r.t. mat_raw, or NULL (needs
 *           mat_raw and per-id materials; RTC_ERR_UNSUPPORTED with
 *           per-interaction materials)
 * The workspace, rtc_workspace_size(RTC_OP_TRACE_FIELDS_ADJOINT_PAT, ...),
 * is required whenever a per-id, Tx or pattern gradient is asked for.  All
 * reductions are in FP64 in a fixed order.  Where the diffuse field is zero
 * (f_s = 0) the pattern gradient is 0. */
rtc_status rtc_trace_fields_adjoint_pat(const rtc_radio* radio, const rtc_paths* paths,
                                        const rtc_materials* mats, const rtc_patterns* pats,
                                        const void* dLda, float* dLd_raw, float* dLd_inter,
                                        float* dLd_tx, float* dLd_pat, void* ws, size_t ws_bytes,
                                        void* stream);

/* Material embeddings (Sec. III-C, Eqs. trainable_materials_1-4): every
 * material m has four embeddings w_1 .. w_4 in R^L, and one read-out vector
 * v in R^L is shared by all materials; u_{m,j} = v . w_{m,j} gives
 * sigma = e^{u_1}, eps_r = 1 + e^{u_2}, S = logistic(u_3), K_x = logistic(u_4).
 *   v  float [L], W float [n_mat, 4, L] row-major, W[m, j-1, :] = w_j of
 *      material m (paper order: sigma, eps_r, S, K_x); 1 <= n_mat <= 4096,
 *      1 <= L <= 1024
 *   raw     float [n_mat * 3], the per-id layout of rtc_materials:
 *           raw[3m] = u_2 (eps_r), raw[3m+1] = u_1 (sigma), raw[3m+2] = u_3 (S)
 *   pat_raw float [n_mat * 6] (rtc_patterns.mat_raw) or NULL:
 *           pat_raw[6m] = u_4 (the K_x logit); its other columns are not touched
 * Each u is an FP64 sum rounded once to float. */
rtc_status rtc_embed_readout(int32_t n_mat, int32_t L, const float* v, const float* W, float* raw,
                             float* pat_raw, void* stream);

/* Backward of rtc_embed_readout: dLd_raw float [n_mat * 3] (required) and
 * dLd_pat float [n_mat * 6] or NULL (only column 0, dL/du_4, is read; NULL
 * counts as 0) give dL/du; writes dLd_v float [L] = sum_{m,j} W[m,j,:] dL/du_{m,j}
 * (FP64 sums in a fixed order) and dLd_W float [n_mat, 4, L] = v dL/du_{m,j}.
 * Outputs are overwritten; either may be NULL. */
rtc_status rtc_embed_readout_backward(int32_t n_mat, int32_t L, const float* v, const float* W,
                                      const float* dLd_raw, const float* dLd_pat, float* dLd_v,
                                      float* dLd_W, void* stream);

/* Neural materials (Sec. III-D): per point p, p_bar = (p - aabb_center) *
 * inv_extent (inv_extent = 1 / longest edge of the scene's axis-aligned
 * bounding box, so p_bar lies in [-1/2, 1/2]^3); input features
 * [p_bar, then for each coordinate and k = 1..n_freq: sin(2^k pi p_bar),
 * cos(2^k pi p_bar)] (the positional encoding of Eq. pos_encoding plus the
 * raw coordinates, 51 features for n_freq = 8); n_hidden ReLU layers of
 * `width`; 3 outputs o mapped to eps_r = 1 + softplus(o0), sigma =
 * softplus(o1), S = logistic(o2).  Weights and layer inputs are rounded to
 * BF16 (nearest even), products accumulate in FP32, biases and output
 * transforms are FP32.  params: FP32 master vector of rtc_mlp_n_params()
 * values, packed W0 [128][51], b0 [128], W1..W3 [128][128] each followed by
 * its bias [128], W4 [3][128], b4 [3] (row-major, out x in).  This build
 * implements n_freq = 8, width = 128, n_hidden = 4. */
typedef struct {
  const float* params;
  float aabb_center[3];
  float inv_extent;
  int32_t n_freq;
  int32_t width;
  int32_t n_hidden;
} rtc_mlp;

int32_t rtc_mlp_n_params(void);
/* Bytes of the buffer rtc_mlp_forward saves for rtc_mlp_backward (its
 * layout is internal to the library). */
size_t rtc_mlp_saved_size(int64_t n_points);
/* Bytes of workspace rtc_mlp_forward (>= the packed weights) and
 * rtc_mlp_backward need; the same buffer serves both. */
size_t rtc_mlp_workspace_size(int64_t n_points);

/* Forward over n_points points (px, py, pz: float [n_points] each, for
 * example the interaction rows of a path store).  out: float [3*n_points],
 * rows eps_r, sigma, S -- the per-interaction material layout of
 * rtc_materials.per_inter.  saved: device buffer of rtc_mlp_saved_size
 * bytes for the backward, or NULL. */
rtc_status rtc_mlp_forward(const rtc_mlp* net, int64_t n_points, const float* px,
                           const float* py, const float* pz, float* out, void* saved,
                           size_t saved_bytes, void* ws, size_t ws_bytes, void* stream);

/* Backward: dLdout float [3*n_points] (rows dL/d eps_r, dL/d sigma, dL/d S,
 * as rtc_trace_fields_adjoint writes them) and the forward's saved buffer ->
 * dLdparams float [rtc_mlp_n_params()] (overwritten).  Weight gradients are
 * summed over points in fixed blocks of 128 and the blocks' partial sums in a
 * fixed order, so the result depends only on the inputs. */
rtc_status rtc_mlp_backward(const rtc_mlp* net, int64_t n_points, const float* dLdout,
                            const void* saved, float* dLdparams, void* ws, size_t ws_bytes,
                            void* stream);

/* Adam step (the optimiser the paper uses, Sec. III-G / IV-B) on float32
 * arrays of length n, in place:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2
 *   p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * step t >= 1. */
rtc_status rtc_adam_step(float* param, const float* grad, float* m, float* v, int64_t n,
                         int32_t step, float lr, float beta1, float beta2, float eps,
                         void* stream);

/* rtc_adam_step with the step count in device memory, for callers that
 * record the calibration step into a HIP graph: step is a device int32
 * holding the number of updates already made; this update uses t = *step + 1
 * in its bias corrections, and with advance != 0 a kernel ordered after the
 * update increments *step (several parameter groups of one optimiser step
 * pass advance = 0 but in the last call).  No host synchronisation, no
 * allocation, no memset. */
rtc_status rtc_adam_step_dev(float* param, const float* grad, float* m, float* v, int64_t n,
                             int32_t* step, int32_t advance, float lr, float beta1, float beta2,
                             float eps, void* stream);

/* y[i] += alpha * x[i] for float32 arrays of length n: accumulation of
 * gradients over batches that one optimiser step streams through (the
 * per-batch entry points overwrite their outputs). */
rtc_status rtc_axpy(float* y, const float* x, float alpha, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RTCAL_H */
