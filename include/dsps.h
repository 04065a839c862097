/*
 * dsps.h -- C ABI of libdsps, the MI355X (gfx950) hot path of differentiable
 * stellar population synthesis (Hearin et al., arXiv 2112.06830).
 *
 * For every galaxy of a population the library turns a tabulated star-
 * formation history, an age-dependent metallicity distribution and dust
 * parameters into apparent AB magnitudes through a set of filters:
 *
 *   age-bin masses from the cumulative SFH     (Section 3.1, Eqs. cspsum, mstartot)
 *   x triweight metallicity weights            (Section 3.2.2, Eq. agedep_mdf;
 *                                               Appendix B, Eqs. triweight, terf)
 *   contracted against the SSP block           (Section 2.1, Eqs. cspdeftheta, full_mdf)
 *   x dust attenuation                         (Section 3.4, Eqs. attenuation-uvbump)
 *   -> redshifted filter integrals, AB mags    (Section 2.2.1, Eq. restmag)
 *
 * optionally over a third SSP axis, the nebular ionization parameter, with a
 * triweight weight per grid point (Section 3.3, Eq. nebsed), with emission-
 * line equivalent widths of the composite SED (Section 2.2.2, Eq. eqw), and
 * it returns the reverse-mode gradient of the magnitudes (Section 2.1:
 * with the SSP block fixed, every gradient flows through the weights).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: DSPS_OK (0) or a negative dsps_status.  No exception ever
 *    crosses the ABI.  dsps_last_error() gives a thread-local message for the
 *    last failing call.
 *  - Unless stated otherwise, array pointers are DEVICE pointers to
 *    contiguous row-major memory owned by the caller (for example torch
 *    tensors).  The library never frees caller memory, never allocates during
 *    a compute call, and never synchronises the host in a compute call: work
 *    is enqueued on the caller's hipStream_t.  Argument and shape checks run
 *    on the host before any launch; a failed check enqueues nothing.
 *  - Scratch memory comes from a caller-provided workspace whose size
 *    dsps_workspace_size() reports; a smaller workspace is DSPS_ERR_WORKSPACE.
 *    (dsps_mags_noalloc instead uses a fixed array the library holds per
 *    device.)
 *  - Outputs are fully overwritten.  Inputs are const.  n_gal == 0 is a no-op
 *    that returns DSPS_OK.  NaN and Inf inputs are not checked; they
 *    propagate.  A band whose transmission misses the SED grid entirely
 *    yields NaN; a zero numerator yields +Inf.
 *  - Device faults surface as DSPS_ERR_DEVICE at the next call that checks
 *    for launch errors, or at the caller's synchronisation.
 *  - Compute calls on different streams may run concurrently if each has its
 *    own workspace.  Handles are immutable after creation.
 *  - All compute calls must be made with the device current on which the
 *    handles were created.
 */
#ifndef DSPS_H
#define DSPS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DSPS_ABI_VERSION 9

typedef enum {
  DSPS_OK = 0,
  DSPS_ERR_ARG = -1,          /* NULL pointer, bad enum or bad scalar        */
  DSPS_ERR_SHAPE = -2,        /* sizes inconsistent or outside the limits    */
  DSPS_ERR_DEVICE = -3,       /* HIP runtime error                           */
  DSPS_ERR_WORKSPACE = -4,    /* workspace too small or misaligned           */
  DSPS_ERR_UNSUPPORTED = -5,  /* valid request the library does not implement */
  DSPS_ERR_ALLOC = -6         /* device allocation failed in a create call   */
} dsps_status;

typedef enum { DSPS_FP32 = 0, DSPS_BF16 = 1 } dsps_precision;

/* Branch order of the k0 attenuation curve (Section 3.4, Eq. kzero).
 * DSPS_K0_SALIM: Leitherer et al. 2002 below 0.15 micron, Calzetti et al. 2000
 * at and above it (the order of the cited Salim et al. parameterisation).
 * DSPS_K0_PRINTED: the order printed in Eq. kzero (Calzetti below). */
typedef enum { DSPS_K0_SALIM = 0, DSPS_K0_PRINTED = 1 } dsps_k0_reading;

/* Extra bit of dsps_ssp_create's precisions mask (see there). */
#define DSPS_SSP_AGE_MAJOR 4

typedef enum {
  DSPS_OP_WEIGHTS = 0, DSPS_OP_SED = 1, DSPS_OP_MAGS = 2, DSPS_OP_MAGS_VJP = 3
} dsps_op;

/* Limits of the library. */
#define DSPS_MAX_MET 16       /* metallicities in the SSP block             */
#define DSPS_MAX_AGE 96       /* ages in the SSP block                      */
#define DSPS_MAX_BAND 8       /* filters per filter set                     */
#define DSPS_MAX_NT 2048      /* points of the tabulated SFH                */
#define DSPS_MAX_FILTER_FLOATS 8192  /* n_band * n_pts of a filter set          */
#define DSPS_MAX_ION 16       /* points of the ionization axis              */
#define DSPS_MAX_LINES 16     /* emission lines per dsps_eqw call           */

/* ---------------------------------------------------------------------------
 * Resident SSP block (Section 2.1: the SSP spectra are loaded once as a
 * contiguous block and then held fixed).
 *
 * dsps_ssp_create copies the block to the current device and prepares it:
 * a wavelength-major, zero-padded float32 copy and, if requested, a bfloat16
 * copy with one power-of-two float32 scale per (metallicity, age) row (the
 * same rows dsps_quantize_bf16 produces), plus per-wavelength attenuation
 * constants for the chosen k0 reading.
 *   n_met, n_age, n_wave   grid sizes; 1 <= n_met <= 16, 1 <= n_age <= 96,
 *                          2 <= n_wave
 *   lgz    HOST [n_met]    log10 Z, strictly ascending
 *   lg_age HOST [n_age]    log10 of the SSP age in years, strictly ascending
 *   wave   HOST [n_wave]   rest-frame wavelength in Angstrom, strictly ascending
 *   lum    HOST [n_met*n_age*n_wave] float32, L_sun/Hz per M_sun formed, row
 *                          (met, age) major, finite and >= 0
 *   precisions             bit mask of (1 << DSPS_FP32) | (1 << DSPS_BF16),
 *                          optionally | DSPS_SSP_AGE_MAJOR: also an age-major
 *                          float32 copy, which dsps_mags needs for the
 *                          age-dependent attenuation (dsps_pop.av_old)
 *   k0_reading             dsps_k0_reading
 *   out                    receives the handle; unchanged on failure
 * Allocates device memory (the only allocating call besides
 * dsps_filters_create); synchronous.  Free with dsps_ssp_destroy.
 * ------------------------------------------------------------------------ */
typedef struct dsps_ssp_s dsps_ssp;
int dsps_ssp_create(int n_met, int n_age, int n_wave, const double *lgz,
                    const double *lg_age, const double *wave, const float *lum,
                    int precisions, int k0_reading, dsps_ssp **out);

/* SSP block with the nebular ionization axis u = log10 U_s (Section 3.3,
 * Eq. nebsed): L_SSP(lambda | tau_i, Z_j, u_k).
 *   n_u     1 <= n_u <= 16 ionization points
 *   lgu     HOST [n_u] log10 U_s, strictly ascending
 *   lum     HOST [n_met*n_age*n_u*n_wave] float32, row (met, age, u) major
 *   precisions  (1 << DSPS_FP32) only when n_u > 1 (the axis is supported
 *           in float32), else as dsps_ssp_create
 * Other arguments as dsps_ssp_create.  Ionization bins are bounded by the
 * midpoints of adjacent grid values (-inf and +inf outermost); the weight of
 * point k is the triweight mass of the galaxy's distribution inside bin k
 * (dsps_pop.lgu, sigma_u).  dsps_sed and dsps_mags (float32) sum over the
 * axis; dsps_weights returns the (metallicity, age) weights without the
 * ionization factor; dsps_mags_vjp adds the gradients w.r.t. the ionization
 * centre and width.  n_u == 1 is dsps_ssp_create. */
int dsps_ssp_create_neb(int n_met, int n_age, int n_u, int n_wave, const double *lgz,
                        const double *lg_age, const double *lgu, const double *wave,
                        const float *lum, int precisions, int k0_reading, dsps_ssp **out);
void dsps_ssp_destroy(dsps_ssp *ssp);

/* ---------------------------------------------------------------------------
 * Resident filter set (Section 2.2.1, T_Q in Eq. restmag).
 *   n_band  1..8 filters;  n_pts >= 2 points per filter, n_band * n_pts <= 8192
 *   wave  HOST [n_band*n_pts] observed-frame Angstrom; each row uniformly
 *         spaced and ascending (relative deviation <= 1e-9), else
 *         DSPS_ERR_UNSUPPORTED
 *   trans HOST [n_band*n_pts] transmission probability, finite and >= 0
 * The transmission at an observed wavelength is the linear interpolation of
 * the table, and zero outside it.  Allocates; synchronous.
 * ------------------------------------------------------------------------ */
typedef struct dsps_filters_s dsps_filters;
int dsps_filters_create(int n_band, int n_pts, const double *wave, const double *trans,
                        dsps_filters **out);
void dsps_filters_destroy(dsps_filters *filters);

/* Flat wCDM cosmology (Section 2.2.1, distance modulus after Eq. restmag).
 * om0 in (0, 1]; h > 0; w0 < 0 (w0 = -1 is LCDM; the age t(z) then uses
 * its closed form, otherwise quadrature). */
typedef struct { double om0, w0, h; } dsps_cosmo;

/* ---------------------------------------------------------------------------
 * A population (structure of arrays, all DEVICE pointers).
 *   n_gal       >= 0 galaxies;  n_t  2..2048 points of the SFH table
 *   t_table     [n_t] cosmic time in Gyr, strictly ascending, shared by all
 *               galaxies; no star forms before t_table[0] and the SFR is
 *               taken as zero after t_table[n_t-1]
 *   sfr         [n_gal*n_t] SFR in M_sun/yr, or NULL when sfh_params is set
 *   sfh_params  [5*n_gal] rows (A, tau, alpha, q, t_q) of the parametric
 *               history SFR(t) = A (t/tau)^alpha exp(-t/tau)
 *               (1 - q Phi((t - t_q)/0.5 Gyr)), or NULL when sfr is set.
 *               Exactly one of sfr and sfh_params is non-NULL.
 *   z           [n_gal] observed redshift, >= 0
 *   lgmet       [n_gal] MDF centre log10 Z at the pivot age
 *   sigma_z     [n_gal] MDF width in dex, > 0
 *   av, delta, bump [n_gal] attenuation A_V, power-law slope, Drude amplitude
 *   lgmet_slope, lg_age_pivot  mu(tau) = lgmet + slope (log10 tau - pivot)
 *   lgmet_old   [n_gal] old-age MDF centre, or NULL.  When set, the centre
 *               moves from lgmet (young) to lgmet_old (old) with the
 *               cumulative triweight of log10 age (Section 3.2.2, Eq.
 *               agedep_mdf with Appendix B, Eq. terf):
 *               mu(tau) = lgmet + (lgmet_old - lgmet)
 *                         T_erf((log10 tau - lg_age_pivot) / mdf_width),
 *               and lgmet_slope is unused
 *   mdf_width   transition width in dex (> 0, finite) when lgmet_old is set;
 *               the transition spans +-3 widths around lg_age_pivot
 *   av_old, delta_old  [n_gal] old-star attenuation parameters, both or
 *               neither.  When set, the attenuation depends on stellar age
 *               (Section 3.4.1, Eq. agedep_dust_csp): A_V and delta of age
 *               tau are av + (av_old - av) T_erf((log10 tau - dust_pivot) /
 *               dust_width) (the old values where T_erf is 1), and likewise
 *               for delta; bump stays age-independent.  dsps_mags,
 *               dsps_sed (apply_dust) and dsps_eqw_pop support it (float32,
 *               on an SSP handle created with DSPS_SSP_AGE_MAJOR, without an
 *               ionization axis), and so does dsps_mags_vjp (av_old_bar, delta_old_bar).
 *   dust_pivot, dust_width  transition centre (log10 yr) and width (dex, > 0)
 *   lgu, sigma_u  [n_gal] centre log10 U_s and width (dex, > 0) of the
 *               triweight ionization distribution (Section 3.3, Eq. nebsed);
 *               required when the SSP handle has n_u > 1, ignored when it
 *               has one ionization point (all weight lands on it)
 *   n_live      DEVICE pointer to one int, or NULL (all n_gal galaxies are
 *               live).  Galaxies with index >= *n_live (clamped to
 *               [0, n_gal]) are padding: no kernel reads their inputs and
 *               their rows of every output are left as they were; the live
 *               galaxies' results are bit for bit those of a call with
 *               n_gal = *n_live.  The count is read on the device when the
 *               kernels run, so a captured graph sized for n_gal serves any
 *               smaller batch (n_gal only bounds the launch grids and the
 *               workspace).  Honoured by dsps_weights, dsps_sed,
 *               dsps_sed_ion_tangent, dsps_mags, dsps_mags_noalloc,
 *               dsps_mags_ion_tangent, dsps_mags_vjp and
 *               dsps_mags_residual_vjp; dsps_eqw_pop refuses a population
 *               that sets it (DSPS_ERR_UNSUPPORTED).
 * ------------------------------------------------------------------------ */
typedef struct {
  int n_gal, n_t;
  const double *t_table;
  const double *sfr;
  const double *sfh_params;
  const float *z, *lgmet, *sigma_z, *av, *delta, *bump;
  double lgmet_slope, lg_age_pivot;
  const float *lgmet_old;
  double mdf_width;
  const float *av_old, *delta_old;
  double dust_pivot, dust_width;
  const float *lgu, *sigma_u;
  const int *n_live;
} dsps_pop;

/* Workspace bytes a call of kind `op` needs for this population shape and
 * precision (filters may be NULL for DSPS_OP_WEIGHTS and DSPS_OP_SED).  The
 * workspace pointer must be 256-byte aligned. */
int dsps_workspace_size(int op, const dsps_ssp *ssp, const dsps_filters *filters,
                        int n_gal, int n_t, int precision, size_t *bytes);

/* ---------------------------------------------------------------------------
 * a0. Parametric SFH table (the stand-in for Diffstar, Section 3.1, Eq.
 * diffstar): sfr[g*n_t + n] = SFR(t_table[n]) for params [5*n_gal] as in
 * dsps_pop.  All DEVICE pointers; float64.
 * ------------------------------------------------------------------------ */
int dsps_sfh_table(const double *t_table, int n_t, const double *sfh_params, int n_gal,
                   double *sfr, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * a1-a4. SSP weights (Eqs. cspsum, mstartot, agedep_mdf).
 *   w      [n_gal*n_met*n_age] float32, M_sun formed per (metallicity, age)
 *          bin, row (g, met, age) major: the age-bin mass times the
 *          metallicity weight.  Age-bin masses are differences of the float64
 *          cumulative trapezoid of the SFR; bins are bounded by geometric
 *          midpoints of adjacent SSP ages (0 and +inf outermost), metallicity
 *          bins by midpoints of adjacent log10 Z (-inf and +inf outermost).
 *   mstar  [n_gal] float64 total mass formed up to t(z), or NULL
 *   workspace  dsps_workspace_size(DSPS_OP_WEIGHTS, ...) bytes (the cosmic
 *          time at each galaxy's redshift)
 * ------------------------------------------------------------------------ */
int dsps_weights(const dsps_ssp *ssp, const dsps_cosmo *cosmo, const dsps_pop *pop,
                 float *w, double *mstar, void *workspace, size_t workspace_bytes,
                 hipStream_t stream);

/* ---------------------------------------------------------------------------
 * a5 (+a6). Composite rest-frame SED (Eqs. cspdeftheta, full_mdf), optionally
 * attenuated (Eq. attenuation).
 *   apply_dust  0 or 1;  precision  dsps_precision
 *   sed   [n_gal*n_wave] float32, L_sun/Hz, rest frame
 * ------------------------------------------------------------------------ */
int dsps_sed(const dsps_ssp *ssp, const dsps_cosmo *cosmo, const dsps_pop *pop,
             int apply_dust, int precision, float *sed, void *workspace,
             size_t workspace_bytes, hipStream_t stream);

/* Derivative of the (optionally attenuated) SED with respect to each
 * galaxy's ionization centre (wrt 0: pop->lgu) or width (wrt 1: sigma_u)
 * (Section 3.3: the gradients the paper takes of line strengths).  The SED of
 * Eq. nebsed is linear in the ionization weights, so this is the same sum
 * with each weight replaced by its derivative
 *   dP_k/du = -(T(z_{k+1}) - T(z_k)) / sigma,
 *   dP_k/dsigma = -(z_{k+1} T(z_{k+1}) - z_k T(z_k)) / sigma,
 * z_e = (e - u)/sigma at the bin edges, T the triweight density (infinite
 * outer edges contribute nothing).  Requires an SSP handle with n_u > 1
 * (else DSPS_ERR_UNSUPPORTED); float32; workspace as dsps_sed
 * (DSPS_OP_SED).  Each galaxy's SED depends only on its own distribution, so
 * row g is also the gradient of any linear functional of SED row g. */
int dsps_sed_ion_tangent(const dsps_ssp *ssp, const dsps_cosmo *cosmo, const dsps_pop *pop,
                         int apply_dust, int wrt, float *dsed, void *workspace,
                         size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * a1-a7. Fused magnitudes: the SED is contracted, attenuated and integrated
 * through every filter without ever being written to memory.
 *   mags     [n_gal*n_band] float32 apparent AB magnitudes
 *            m = -2.5 log10(num / (AB0 den)) + D_mod(z) - 2.5 log10(1+z);
 *            at z = 0 the absolute magnitude of Eq. restmag (no distance
 *            terms), as for the Section 4.1 population observed at z = 0
 *   bands    [n_gal*2*n_band] float32 (num_b then den_b per galaxy): the two
 *            trapezoid sums of Eq. restmag over the redshifted grid, or NULL.
 *   moments  [n_gal*3*n_band] float32 dust moments of the band sums, or NULL
 *            (DSPS_FP32 only, else DSPS_ERR_UNSUPPORTED): for each band the
 *            sums of Eq. restmag's numerand T q F L times k_lambda, times
 *            k0 (lambda/5500)^delta log2(lambda/5500), and times the bump
 *            profile D(lambda) (Eqs. attenuation-uvbump), in that order.
 * dsps_mags_vjp accepts bands and moments to skip the forward pass.
 * ------------------------------------------------------------------------ */
int dsps_mags(const dsps_ssp *ssp, const dsps_filters *filters, const dsps_cosmo *cosmo,
              const dsps_pop *pop, int precision, float *mags, float *bands, float *moments,
              void *workspace, size_t workspace_bytes, hipStream_t stream);

/* dsps_mags for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results (bit for bit) and errors as dsps_mags, without the
 * workspace: its scratch is a fixed array of DSPS_NOALLOC_SCRATCH_BYTES
 * bytes that the library holds on each device it runs on until the process
 * ends.  The call allocates and frees nothing (kernel instrumentation,
 * dsps_profile_enable, is not recorded for it).  The population runs in as
 * many batches of whole 128-galaxy tiles as the array needs; a population
 * whose per-galaxy arrays alone do not fit beside one tile's batch (about
 * two million galaxies on the 12 x 94 x 5994 grid) is refused with
 * DSPS_ERR_SHAPE before any launch.  Every call on one device shares that
 * device's array: calls that overlap in time on one device (on different
 * streams, or from different threads) race and give undefined results;
 * calls in stream order on one stream are safe.  The array's contents from
 * an earlier call are never read. */
#define DSPS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int dsps_mags_noalloc(const dsps_ssp *ssp, const dsps_filters *filters, const dsps_cosmo *cosmo,
                      const dsps_pop *pop, int precision, float *mags, float *bands,
                      float *moments, hipStream_t stream);

/* Derivative of the float32 magnitudes with respect to each galaxy's
 * ionization centre (wrt 0: pop->lgu) or width (wrt 1: sigma_u) (Section 3.3,
 * Eq. nebsed): the fused contraction runs with the ionization weights
 * replaced by their derivatives (as dsps_sed_ion_tangent), giving the band
 * sums' derivatives dnum_b, and dm_b = -2.5 / ln 10 dnum_b / num_b.
 *   bands   [n_gal*2*n_band] from dsps_mags with the same inputs, or NULL (the
 *           forward pass then runs first, in the workspace)
 *   dmags   [n_gal*n_band] float32, device
 * Each galaxy's magnitudes depend only on its own distribution, so dmags is
 * also the per-galaxy gradient; a cotangent m_bar gives
 * lgu_bar[g] = sum_b m_bar[g, b] dmags[g, b].  Requires n_u > 1; workspace
 * as dsps_mags (DSPS_OP_MAGS); no age-dependent attenuation. */
int dsps_mags_ion_tangent(const dsps_ssp *ssp, const dsps_filters *filters,
                          const dsps_cosmo *cosmo, const dsps_pop *pop, int wrt,
                          const float *bands, float *dmags, void *workspace,
                          size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * a9. Vector-Jacobian product of dsps_mags (reverse mode).
 *   mags_bar        [n_gal*n_band] float32 cotangent of the magnitudes
 *   bands, moments  from dsps_mags with the same inputs in DSPS_FP32, or both
 *                   NULL (then the forward pass runs first, in the workspace)
 *   sfr_bar         [n_gal*n_t] float64 gradient w.r.t. the SFR table, or NULL
 *   sfh_params_bar  [5*n_gal] float64 gradient w.r.t. (A, tau, alpha, q, t_q);
 *                   requires pop->sfh_params, else NULL
 *   lgmet_bar, lgmet_old_bar, sigma_bar, av_bar, delta_bar, bump_bar
 *                   [n_gal] float32 each, or NULL (lgmet_old_bar requires
 *                   pop->lgmet_old)
 *   lgu_bar, sigma_u_bar  [n_gal] float32, or NULL: gradients w.r.t. the
 *                   ionization centre and width (SSP handle with n_u > 1,
 *                   else DSPS_ERR_ARG): the transposed contraction also
 *                   returns each ionization point's cotangent
 *                   sum_k W[k] (Lbar . L_u[k]), which the derivatives of the
 *                   ionization weights carry to the centre and width
 *   av_old_bar, delta_old_bar  [n_gal] float32, or NULL: gradients w.r.t. the
 *                   old-star attenuation (requires pop->av_old, else
 *                   DSPS_ERR_ARG)
 * With the age-dependent attenuation (Section 3.4.1, Eq. agedep_dust_csp;
 * float32, an SSP handle created with DSPS_SSP_AGE_MAJOR, no ionization
 * axis) every age has its own F_i: the SED cotangent is taken without the
 * attenuation and the transposed contraction applies F_i per age,
 * Wbar[j, i] = sum_l G F_i L[j, i]; the dust cotangents collect per age
 * (split between the young and old parameters by 1 - T_erf and T_erf), so
 * there are no moments: pass moments = NULL (bands may still be given).
 * With an ionization axis (Section 3.3, Eq. nebsed) the transposed
 * contraction runs once per ionization point a tile's members reach, against
 * that point's block of the adjoint table, each galaxy's SED cotangent scaled
 * by its weight of the point.
 * The dust gradients are the band cotangents applied to the moments; the SED
 * cotangent F q sum_b gamma_b T_b needs no SED, so the backward pass holds no
 * forward contraction.  Redshift gets no gradient.
 * ------------------------------------------------------------------------ */
int dsps_mags_vjp(const dsps_ssp *ssp, const dsps_filters *filters, const dsps_cosmo *cosmo,
                  const dsps_pop *pop, int precision, const float *mags_bar,
                  const float *bands, const float *moments, double *sfr_bar,
                  double *sfh_params_bar, float *lgmet_bar, float *lgmet_old_bar,
                  float *sigma_bar, float *av_bar, float *delta_bar, float *bump_bar,
                  float *av_old_bar, float *delta_old_bar, float *lgu_bar, float *sigma_u_bar,
                  void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Forward magnitudes and the reverse pass of the weighted squared residual
 *   L = sum_g sum_b wt[g, b] (m[g, b] - target[g, b])^2,
 * the chi-square term of the likelihood analyses that gradient-based
 * optimisers and Hamiltonian Monte Carlo evaluate (Section 1), in one call:
 * the ordering sort, the per-galaxy scalars and the weights run once, the
 * forward contraction writes the magnitudes, and the reverse pass takes the
 * cotangent mags_bar = (m - target) * (2 wt), formed in float32 on the device
 * from the magnitudes just computed.
 *   target  [n_gal*n_band] float32 target magnitudes, device
 *   wt      [n_gal*n_band] float32 weights (for example 1 / sigma^2), or NULL
 *           (all 1); a row of zeros removes a galaxy from the loss
 *   mags    [n_gal*n_band] float32 output: the magnitudes, as dsps_mags
 *   gradient outputs as dsps_mags_vjp (any may be NULL)
 *   workspace  dsps_workspace_size(DSPS_OP_MAGS_VJP, ..., DSPS_FP32) bytes
 * Float32 only.  mags and every gradient equal, bit for bit, dsps_mags
 * (DSPS_FP32, with bands and moments) followed by dsps_mags_vjp with that
 * cotangent; errors as those two calls (target NULL: DSPS_ERR_ARG). */
int dsps_mags_residual_vjp(const dsps_ssp *ssp, const dsps_filters *filters,
                           const dsps_cosmo *cosmo, const dsps_pop *pop, const float *target,
                           const float *wt, float *mags, double *sfr_bar, double *sfh_params_bar,
                           float *lgmet_bar, float *lgmet_old_bar, float *sigma_bar,
                           float *av_bar, float *delta_bar, float *bump_bar, float *av_old_bar,
                           float *delta_old_bar, float *lgu_bar, float *sigma_u_bar,
                           void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Emission-line equivalent widths of rest-frame SEDs (Section 2.2.2, Eq. eqw).
 * For each line the continuum L_0 is the least-squares quadratic in
 * (lambda - centre) fitted to the SED at the grid points of the neighbourhood
 * |lambda - centre| <= fit_half_width outside the line window
 * |lambda - centre| <= half_width, every point with equal weight; the width is
 * the trapezoid rule, over the grid points inside the line window, of
 * (L - L_0) / L_0 in rest-frame Angstrom (positive for emission).  The fit and
 * the sums run in float64 on float32 SEDs.
 *   ssp    handle whose wavelength grid the SEDs are on
 *   sed    [n_gal*n_wave] float32, device (e.g. dsps_sed output)
 *   lines  HOST [n_line], 1 <= n_line <= DSPS_MAX_LINES; 0 < half_width <
 *          fit_half_width; the line window must hold >= 2 grid points and the
 *          neighbourhood >= 3 points outside it (else DSPS_ERR_SHAPE)
 *   eqw    [n_gal*n_line] float32, device; a non-positive continuum at a
 *          window point gives Inf or NaN there
 * ------------------------------------------------------------------------ */
typedef struct { double centre, half_width, fit_half_width; } dsps_line;
int dsps_eqw(const dsps_ssp *ssp, const float *sed, int n_gal, const dsps_line *lines,
             int n_line, float *eqw, hipStream_t stream);
/* The widths and their tangent along an SED tangent dsed [n_gal*n_wave]
 * (e.g. dsps_sed_ion_tangent): the continuum fit is linear, so its tangent
 * is the same fit of dsed, and the integrand's tangent is
 * (dL L_0 - L dL_0) / L_0^2.  deqw [n_gal*n_line] float32, device. */
int dsps_eqw_jvp(const dsps_ssp *ssp, const float *sed, const float *dsed, int n_gal,
                 const dsps_line *lines, int n_line, float *eqw, float *deqw,
                 hipStream_t stream);
/* Equivalent widths straight from a population, without the SED in memory:
 * the (optionally attenuated) SED contraction of dsps_sed runs only on the
 * 128-point wavelength chunks the lines' neighbourhoods touch (at most 64 in
 * all, else DSPS_ERR_SHAPE), into workspace rows, and the widths follow as in
 * dsps_eqw.  Every width equals dsps_eqw on dsps_sed's output bit for bit.
 *   wrt    -1: widths only; 0 / 1: also their derivative in each galaxy's
 *          ionization centre / width (as dsps_sed_ion_tangent then
 *          dsps_eqw_jvp; SSP handle with n_u > 1)
 *   eqw, deqw  [n_gal*n_line] float32, device (deqw only with wrt >= 0)
 *   workspace  dsps_eqw_pop_workspace() bytes
 * Float32; the handle needs the float32 table. */
int dsps_eqw_pop_workspace(const dsps_ssp *ssp, int n_gal, const dsps_line *lines, int n_line,
                           int wrt, size_t *bytes);
int dsps_eqw_pop(const dsps_ssp *ssp, const dsps_cosmo *cosmo, const dsps_pop *pop,
                 int apply_dust, const dsps_line *lines, int n_line, int wrt, float *eqw,
                 float *deqw, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Population summary of the Section 4.1 forward model: a red-colour cut and
 * a histogram of one band's magnitude over the selected galaxies, smoothed
 * with the triweight of Appendix B (Eqs. triweight, terf) so that gradients
 * reach every galaxy:
 *   w_g    = T_erf((c_g - colour_cut) / colour_width),   c_g = m_a - m_b
 *   B_k(m) = T_erf((e_{k+1} - m) / mag_width) - T_erf((e_k - m) / mag_width)
 *   hist_k = sum_g w_g B_k(m_g, band_m)
 * with T_erf the cumulative triweight (support +-3 widths).  A zero width
 * gives the hard cut (c > colour_cut) or the plain histogram with bins
 * [e_k, e_{k+1}), the last closed on the right.  A galaxy whose colour or
 * magnitude is not finite contributes nothing.
 *   mags       [n_gal*n_band] float32, device (e.g. dsps_mags output)
 *   band_a, band_b, band_m   band indices in [0, n_band)
 *   colour_width, mag_width  >= 0, finite
 *   edges      [n_bins+1] float64, device, strictly ascending (not checked);
 *              1 <= n_bins <= DSPS_MAX_SUMMARY_BINS
 *   hist       [n_bins] float64, device.  Partial sums are reduced in a
 *              fixed order, so the result is deterministic.
 *   workspace  dsps_pop_summary_workspace() bytes, device
 * dsps_pop_summary_vjp writes mags_bar [n_gal*n_band] float32 (every entry),
 * the gradient of sum_k hist_bar[k] hist_k (hist_bar float64, device); it is
 * zero for zero widths (the hard summary is piecewise constant) and for
 * galaxies that contribute nothing.
 * ------------------------------------------------------------------------ */
#define DSPS_MAX_SUMMARY_BINS 4096
int dsps_pop_summary_workspace(int n_gal, int n_bins, size_t *bytes);
int dsps_pop_summary(const float *mags, int n_gal, int n_band, int band_a, int band_b,
                     double colour_cut, double colour_width, int band_m, const double *edges,
                     int n_bins, double mag_width, double *hist, void *workspace,
                     size_t workspace_bytes, hipStream_t stream);
int dsps_pop_summary_vjp(const float *mags, int n_gal, int n_band, int band_a, int band_b,
                         double colour_cut, double colour_width, int band_m,
                         const double *edges, int n_bins, double mag_width,
                         const double *hist_bar, float *mags_bar, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * a8. BF16 quantisation with power-of-two row scales.
 *   x      [rows*cols] float32, finite
 *   q      [rows*cols] bfloat16 bits: round-to-nearest-even of x / scale[row]
 *   scale  [rows] float32, the smallest power of two >= max(x[row]) (1 for an
 *          all-zero row)
 * ------------------------------------------------------------------------ */
int dsps_quantize_bf16(const float *x, int rows, int cols, uint16_t *q, float *scale,
                       hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Instrumentation.  While enabled, every kernel launch of the compute calls
 * is bracketed by HIP events recorded on the caller's stream (process-wide,
 * thread-safe).  dsps_profile_enable(1) clears earlier records;
 * dsps_profile_read waits for the recorded events of one kernel and returns
 * their summed duration in milliseconds and the number of launches.  Not
 * usable under stream capture.
 * ------------------------------------------------------------------------ */
typedef enum {
  DSPS_KERNEL_WEIGHTS = 0,      /* per-galaxy scalars, age masses, W rows   */
  DSPS_KERNEL_MAGS_GEMM = 1,    /* fused contraction + attenuation + filters */
  DSPS_KERNEL_MAGS_FINALIZE = 2,
  DSPS_KERNEL_ZSORT = 3,
  DSPS_KERNEL_SED_GEMM = 4,
  DSPS_KERNEL_VJP_LBAR = 5,     /* adjoint: SED cotangent over tile windows  */
  DSPS_KERNEL_VJP_WBAR = 6,     /* adjoint: transposed contraction          */
  DSPS_KERNEL_VJP_WEIGHTS = 7,  /* adjoint: weights -> SFH, MDF parameters  */
  DSPS_KERNEL_SUMMARY = 8,      /* population summary (partials + reduction) */
  DSPS_KERNEL_EQW = 9,          /* emission-line equivalent widths          */
  DSPS_KERNEL_COUNT = 10
} dsps_kernel_id;
int dsps_profile_enable(int on);
int dsps_profile_read(int kernel_id, double *total_ms, int *launches);

/* Introspection. */
int dsps_abi_version(void);
const char *dsps_last_error(void);
/* Grid sizes of a handle: n_met, n_age, n_wave, precisions, k0_reading. */
int dsps_ssp_info(const dsps_ssp *ssp, int *n_met, int *n_age, int *n_wave,
                  int *precisions, int *k0_reading);
/* Points of the ionization axis (1 for a block without it). */
int dsps_ssp_ion_info(const dsps_ssp *ssp, int *n_u);
int dsps_filters_info(const dsps_filters *filters, int *n_band, int *n_pts);

#ifdef __cplusplus
}
#endif

#endif /* DSPS_H */
