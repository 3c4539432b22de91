/*
 * dsl.h - C ABI of the MI355X dark-siren population log-likelihood library.
 *
 * The library evaluates, for a batch of B hyperparameter points Lambda, the
 * hierarchical dark-siren log-likelihood of a catalogue of gravitational-wave
 * events (paper: Sec. II A, Eqs. 3-5, 7 and 8):
 *
 *   ln L(Lambda) = sum_i ln L_i - N_det ln alpha,
 *   L_i   = (1/N_s,i) sum over the pixels j of event i that pass the
 *           effective-sample-size gate (Eq. 8) of sum_k w_k,
 *   alpha = (1/N_draw) sum over detected injections n of w_n,
 *   w     = p_LOS(z) psi(z)/(1+z) p1(m1) p2(m2|m1)
 *           / ( |d(m1_det, m2_det, d_L)/d(m1, m2, z)| * pi ),
 *
 * where z is the flat-LambdaCDM redshift of each sample's luminosity distance
 * (Eq. 1), p_LOS the sample's pixel redshift prior (Eq. 5; the sky-averaged
 * table for injections), pi the parameter-estimation prior (Eq. 7; the draw
 * density for injections), p1/p2 the MultiPeak mass model and psi the
 * Madau-Dickinson rate shape named in Appendix A.  N_det is the number of
 * events (Eq. 3 with the scale-free rate prior of Sec. II A).
 *
 * Hyperparameter layout (16 doubles per point, in this order):
 *   H0 [km/s/Mpc], Omega_m, alpha, beta, m_min, m_max, delta_m,
 *   mu_low, sigma_low, mu_high, sigma_high, lambda_g, lambda_low,
 *   gamma, kappa, z_p                       (Appendix A, Table II)
 *
 * Conventions
 *   - Return codes: DSL_OK (0) or one of the DSL_E* codes; the message of the
 *     last failure on the calling thread is returned by dsl_last_error().
 *   - A Lambda outside the model's domain is not an error: its ln L is -inf
 *     and flag bit DSL_FLAG_INVALID_LAMBDA is set (see the flag list below).
 *   - Pointers named d_* are device pointers (memory of the device that was
 *     current when the handle was created); every other pointer is a host
 *     pointer.  Device outputs are owned by the caller.
 *   - Work is enqueued on the given HIP stream (NULL = the default stream)
 *     and is asynchronous: results are valid once the stream has reached
 *     them.  A handle owns one workspace, so calls on one handle must not
 *     overlap in time (use one handle per concurrent stream).
 */
#ifndef DSL_H
#define DSL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DSL_N_LAMBDA 16

enum {
  DSL_OK = 0,
  DSL_EINVAL = 1,   /* bad argument or malformed catalogue */
  DSL_ENOMEM = 2,   /* device or host allocation failed */
  DSL_EHIP = 3,     /* HIP runtime error (message carries the HIP error) */
  DSL_ESTATE = 4    /* handle not usable (e.g. destroyed, wrong device) */
};

/* Per-Lambda flag bits written to d_flags. */
enum {
  DSL_FLAG_INVALID_LAMBDA = 1u, /* Lambda outside the domain (H0 <= 0, Omega_m not in [0,1],
                                   m_min <= 0 or >= m_max, delta_m < 0, sigma <= 0,
                                   lambda not in [0,1], z_p <= -1, non-finite) */
  DSL_FLAG_EVENT_NO_PIXEL = 2u, /* some event has no pixel passing the N_eff gate */
  DSL_FLAG_ALPHA_ZERO = 4u,     /* every injection weight is zero */
  DSL_FLAG_NONFINITE = 8u       /* a non-finite intermediate was met */
};

enum { DSL_PRECISION_FP64 = 0, DSL_PRECISION_FP32 = 1 };

/*
 * Catalogue description (all host pointers; read during dsl_create only).
 *
 * CSR layout (the padded (event, pixel, sample) tensor of Sec. II B made
 * ragged, as its conclusions propose):
 *   event_pix_off[n_events+1]  pixels of event i are [event_pix_off[i], event_pix_off[i+1])
 *   pix_samp_off[n_pix+1]      samples of pixel j are [pix_samp_off[j], pix_samp_off[j+1])
 *   pix_los_row[n_pix]         row of `los` holding pixel j's redshift prior
 *   los[n_los_rows * n_z]      redshift prior tables, row-major, on n_z uniform
 *                              nodes over [0, z_max] (linearly interpolated, zero outside)
 *   sky_z[n_z]                 sky-averaged redshift prior (selection term)
 * The tables are given either in float32 (los, sky_z) or in float64 (los_f64,
 * sky_z_f64): exactly one pointer of each pair is non-NULL.  They are converted
 * at upload to the precision of the handle (float32 for DSL_PRECISION_FP32,
 * float64 for DSL_PRECISION_FP64), so an FP64 handle keeps float64 tables.
 * Samples (n_samp, detector frame): m1d, m2d [Msun], dl [Mpc], ln_pi (ln of the
 * PE prior density in (m1_det, m2_det, d_L)).  Injections (n_inj detected out of
 * n_draw drawn): the same with ln_pdraw, the ln of the draw density.
 * Requirements: offsets start at 0, are non-decreasing and end at n_pix / n_samp;
 * 0 <= pix_los_row < n_los_rows; 2 <= n_z <= 2^24; z_max > 0; masses and
 * distances finite and > 0; ln_pi / ln_pdraw finite; los and sky_z finite and
 * >= 0; n_draw >= n_inj >= 1; 1 <= n_events < 2^31 - 1; n_pix < 2^31 - 1.
 * Violations return DSL_EINVAL.
 */
typedef struct dsl_catalog_desc {
  int64_t n_events;
  const int64_t* event_pix_off;
  int64_t n_pix;
  const int64_t* pix_samp_off;
  const int32_t* pix_los_row;
  int64_t n_los_rows;
  int32_t n_z;
  double z_max;
  const float* los;        /* float32 tables, or NULL when los_f64 is given */
  const float* sky_z;      /* float32 sky table, or NULL when sky_z_f64 is given */
  const double* los_f64;   /* float64 tables, or NULL when los is given */
  const double* sky_z_f64; /* float64 sky table, or NULL when sky_z is given */
  int64_t n_samp;
  const double* m1d;
  const double* m2d;
  const double* dl;
  const double* ln_pi;
  int64_t n_inj;
  const double* inj_m1d;
  const double* inj_m2d;
  const double* inj_dl;
  const double* inj_ln_pdraw;
  int64_t n_draw;
  int32_t precision; /* DSL_PRECISION_FP64 or DSL_PRECISION_FP32 (FP32 weights, FP64 sums) */
  /* Per-pixel random downsampling at upload (Sec. II C, "Memory Reduction
   * Strategies"): when > 0, a pixel with more samples keeps exactly this many,
   * those with the smallest keys splitmix64(seed + splitmix64(pixel << 32 | k))
   * (k = position in the pixel; ties by k), in their original order.  N_s,i
   * becomes the number of kept samples.  0 keeps every sample. */
  int64_t max_samples_per_pixel;
  uint64_t downsample_seed;
} dsl_catalog_desc;

typedef struct dsl_handle dsl_handle;

/*
 * Copy a catalogue to the current device and build its work list.
 * The library owns the device copy until dsl_destroy.  *out is NULL on failure.
 */
int dsl_create(const dsl_catalog_desc* desc, dsl_handle** out);

/*
 * Set an option (takes effect on the next call):
 *   "neff_min"   threshold of the pixel gate of Eq. (8), default 2 (ties pass)
 *   "gate_mode"  0 pixel gate (default), 1 also reject events whose N_eff < neff_min,
 *                2 no gate
 *   "z_prior"    0 = each sample's redshift prior is its pixel's LOS table and the
 *                selection term uses sky_z (dark sirens, Eq. 5; default); 1 = every
 *                sample and injection uses the comoving-volume shape
 *                dV_c/dz ∝ I(z)^2/E(z) of the point's Omega_m (spectral sirens,
 *                the setting of the paper's O5 mock analysis); tables are ignored
 *   "numerator"  0 = each pixel contributes the sum of its samples' weights (default);
 *                1 = the paper's KDE form (Eq. 6): the pixel's weighted Gaussian KDE
 *                in redshift, weights of Eq. (7) without prior and rate, times the
 *                pixel's LOS table and psi(z)/(1+z), integrated by the trapezoid rule
 *                on "kde_grid" uniform nodes from max(0, min z - 5h) to
 *                min(z_max, max z + 5h) over the pixel's in-support samples; the gate
 *                of Eq. (8) uses the same weights.  Value only (dsl_loglike_grad
 *                returns DSL_EINVAL) and only with z_prior 0
 *   "kde_bandwidth" 0 Scott 1.06 s n^-1/5 (default), 1 Silverman
 *                0.9 min(s, IQR/1.34) n^-1/5, 2 biweight 1.06 sqrt(midvariance) n^-1/5
 *                (Appendix D), over the pixel's in-support redshifts (unweighted, s with
 *                n - 1, linear quantiles); h = 0 (one sample, equal values, zero MAD)
 *                makes each sample a point mass
 *   "kde_grid"   grid nodes of the KDE numerator, 2 ... 1024 (default 256, Sec. III C)
 *   "max_batch"  largest B accepted (default 4096)
 *   "lambda_tile" Lambda per wavefront for the sweep (0 = automatic; 1, 4, 16, 64)
 *   "chunk"      target samples per work item (0 = automatic)
 *   "timing"     1 = record HIP events around each kernel (see dsl_get_timing)
 *   "graph"      1 = capture each (B, entry point) launch sequence once in a
 *                HIP graph and replay it (default 1)
 * Unknown keys or out-of-range values return DSL_EINVAL.
 */
int dsl_set_option(dsl_handle* h, const char* key, double value);

/* Read back an option or a catalogue size ("n_events", "n_pix", "n_samp",
 * "n_inj", "n_items", "precision", ...), "lambda_tile_used" (the Lambda tile
 * of the last call), "device_bytes" (device memory the handle holds),
 * "work_list_bytes" (of it, the work list: items, order, event offsets, split pixels),
 * "kde_evals" and "kde_nodes" (of the last call with the KDE numerator: the
 * (sample, grid node) kernel terms and the grid nodes evaluated; both wait for
 * the device), "kde_units" (the grid-stage units of that call: n_pix, or more
 * when large pixels were split into parts), or, after a call made with option
 * "timing" = 1, "ms_sweep_only" (the weight sweep alone) and "ms_pixels" (the
 * per-pixel stage after it: the KDE kernel, or the gate of split pixels).
 * Returns DSL_EINVAL for unknown keys. */
int dsl_get_info(dsl_handle* h, const char* key, double* value);

/*
 * Log-likelihood of B points (Sec. II A: Eq. 1 for z(d_L), Eq. 7 for the
 * per-sample weights, Eq. 8 for the pixel gate, Eq. 5 for the per-event Monte
 * Carlo sums and the selection term, Eq. 3 for ln L), one persistent sweep
 * for the whole batch: every sample record is read once for all B points.
 *   d_lambda     [B][16] device, layout above
 *   d_logL       [B] device, ln L (or -inf with a flag)
 *   d_logL_event [B][n_events] device or NULL: ln L_i
 *   d_neff_event [B][n_events] device or NULL: (sum w)^2 / sum w^2 over the
 *                event's passing pixels (0 if none)
 *   d_neff_sel   [B] device or NULL: effective sample size of the injections
 *   d_flags      [B] device or NULL: DSL_FLAG_* bits
 *   stream       hipStream_t (NULL = default stream)
 * 1 <= B <= max_batch, otherwise DSL_EINVAL.
 */
int dsl_loglike(dsl_handle* h, const double* d_lambda, int B, double* d_logL,
                double* d_logL_event, double* d_neff_event, double* d_neff_sel,
                uint32_t* d_flags, void* stream);

/*
 * Log-likelihood and its gradient d ln L / d Lambda (all 16 entries) for B
 * points, by an adjoint sweep that recomputes every per-sample weight and its
 * derivatives (nothing is stored between calls): the derivative of Eq. 3 through
 * Eqs. 5 and 7, with z(d_L) of Eq. 1 differentiated implicitly,
 *   d ln L = sum_i <d ln w>_(w, passing pixels of i) - N_det <d ln w>_(w, injections).
 * Gates and supports are held at their current state (derivative almost
 * everywhere); entries of a point whose ln L is -inf are 0.
 *   d_grad [B][16] device.  Other arguments as in dsl_loglike; the per-event
 *   outputs (d_logL_event, d_neff_event, d_neff_sel) are the same as there.
 */
int dsl_loglike_grad(dsl_handle* h, const double* d_lambda, int B, double* d_logL,
                     double* d_grad, double* d_logL_event, double* d_neff_event,
                     double* d_neff_sel, uint32_t* d_flags, void* stream);

/*
 * dsl_loglike_grad without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving or sampling loops,
 * harnesses that forbid hipMalloc.  Arguments, outputs and results are those of
 * dsl_loglike_grad (Monte Carlo numerator only).  The call allocates nothing,
 * copies nothing from the host and captures no graph: its workspace (per-point
 * tables, per-item partial sums, combine records) lives in one static device
 * array of 64 MiB per GPU, held by the library until the process ends, and the
 * handle's current work list is used as it stands.  A batch whose workspace
 * exceeds 64 MiB returns DSL_EINVAL (e.g. the 5000-event catalogue with 64
 * points needs about 0.75 GB: use dsl_loglike_grad there).  Every call on one
 * GPU shares that array, from every handle: calls that overlap in time on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller; the array keeps the last call's contents (the only part that must
 * start at zero, the work and slice counters, is zeroed by the call itself).
 */
int dsl_loglike_grad_noalloc(dsl_handle* h, const double* d_lambda, int B, double* d_logL,
                             double* d_grad, double* d_logL_event, double* d_neff_event,
                             double* d_neff_sel, uint32_t* d_flags, void* stream);

/*
 * Choose the sweep configuration (Lambda tile, chunk) for batches of B points
 * by timing the candidates on the current device; the choice is cached in the
 * handle and, when cache_path is not NULL, appended to that text file (one
 * line per device/catalogue/options/B key; read first if it exists, and a
 * line whose configuration this library does not launch is ignored).
 */
int dsl_autotune(dsl_handle* h, int B, int with_grad, const char* cache_path);

/*
 * Kernel times of the last call made with option "timing" = 1 (milliseconds,
 * host pointers): setup, sweep, combine.  Waits for that call to finish.
 */
int dsl_get_timing(dsl_handle* h, float* ms_setup, float* ms_sweep, float* ms_combine);

/* Release the handle and its device memory (NULL is ignored). */
void dsl_destroy(dsl_handle* h);

/* Message of the last failure on the calling thread ("" if none). */
const char* dsl_last_error(void);

/* Library version string. */
const char* dsl_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DSL_H */
