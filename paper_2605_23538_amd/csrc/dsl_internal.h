// Internal layouts shared by the host side (dsl_abi.cpp) and the kernels
// (dsl_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsl {

constexpr double C_KMS = 299792.458;
constexpr double LN2 = 0.69314718055994530942;
constexpr double LOG2E = 1.44269504088896340736;

// Hermite segments of the per-Lambda tables.  z(u) is tabulated as z/u against
// v = sqrt(1 + 4u) (see setup kernel); the smoothing-window table as
// rho = Z(m1) / (S(m1) m1^(beta+1)) against t = (m1 - m_min) / delta_m.
constexpr int NU_F32 = 64;
constexpr int NW_F32 = 64;
constexpr int NU_F64 = 1024;
constexpr int NW_F64 = 256;
// The adjoint's window tables (the window-integral parts of d rho/d(beta,
// m_min, delta_m)) use every second node, Hermite with analytic tangents.
constexpr int NWG_F32 = NW_F32 / 2;
constexpr int NWG_F64 = NW_F64 / 2;

// I(z) is tabulated at the starts of KZ_I uniform panels over [0, z_max] and
// at z_max (prefix sums of 8-point Gauss-Legendre), in FP64.
constexpr int KZ_I = 256;
// A sample whose table coordinate z/dz lies within this relative distance of
// a node takes its cell from an FP64 comparison (FP32 redshifts are within
// 3.2e-7 of the FP64 ones): d_L H0/c against U(z_k) = (1+z_k) I(z_k) at the
// node, U increasing, so the cell is the one of the FP64 redshift.
constexpr float NODE_TAU = 8e-7f;

constexpr int R_SENTINEL = -(1 << 20);   // "no weight yet" binary exponent
constexpr int RESCALE_MARGIN = 60;        // new max exponent that forces a rescale

// Per-Lambda constants of the sweep (one copy per precision).
template <typename T>
struct LamC {
  T H0;            // u = (d_L / c) * H0
  T u_max;         // (1+z_max) I(z_max): larger u is outside the support
  T inv_hv;        // table segments per unit of v = sqrt(1 + 4u)
  T Om, OL;        // Omega_m, 1 - Omega_m
  T c0;            // log2(H0 / c)
  T alpha, beta, mmin, mmax, dm, inv_dm;
  T cP, cL, cH;    // log2 of mixture weight x component normalisation
  T muL, kL, muH, kH;   // peak centres, -log2(e) / (2 sigma^2)
  T s, inv_s, lM, zw;   // beta+1, 1/(beta+1), log2(m_min+delta_m), Z_w / M^s
  T inv_M;              // 1/(m_min+delta_m)
  T gm3, gk, Lp;   // gamma - 3, gamma + kappa, log2(1 + z_p)
  // --- gradient constants (natural-log derivatives of the normalisations)
  T dbP_alpha, dbP_mmin, dbP_mmax;            // d ln b_P
  T dbL_mu, dbL_sig, dbL_mmin, dbL_mmax;       // d ln b_L (b_L = 1/(sig sqrt(2pi) dPhi))
  T dbH_mu, dbH_sig, dbH_mmin, dbH_mmax;
  T sigL, sigH;                               // sigma_low, sigma_high
  T lg, ll;                                   // lambda_g, lambda_low
  T zw_beta, zw_mmin, zw_dm;                  // window integrals of d/d(beta, m_min, dm) of m^beta S, / M^s
  T gamma, kappa, inv_opzp;                   // gamma, kappa, 1/(1+z_p)
  T inv_H0;                                   // 1/H0
  T k23, hOm;                                 // (2/3)/(1-Om), 1/(2 Om)
  T isL2, isL3, isH2, isH3;                   // sigma^-2, sigma^-3 of the peaks
  T aPg, aLg, aLl, aHl;                       // 1/(1-lg), 1/lg, 1/ll, 1/(1-ll) (0 at the edges)
  T inv_s2;                                   // 1/(beta+1)^2
  // rounding residuals (x - (T)x) of the constants whose FP32 rounding would
  // shift every sample alike: H0 (through u) and the mass locations m_min,
  // mu_low, mu_high (through the differences m - x); 0 in FP64
  T H0_lo, mmin_lo, muL_lo, muH_lo;
  int om_case;                                // 0 general, 1 Om ~ 0, 2 Om ~ 1
  int valid;
};

// Number of window-derivative tables used by the adjoint (beta, m_min, delta_m).
constexpr int N_WIN_GRAD = 3;
// Per-point FP64 coefficients that map the adjoint's 16 basis sums to the
// gradient (written by setup, applied by combine).
constexpr int N_GMAP = 24;

// Work item: a run of whole pixels of one event, a part of one large pixel
// (pix1 == pix0: samples [s0, s1) of pixel pix0, written ungated), or a run of
// injections (event == -1).
struct WorkItem {
  int32_t event;     // >= 0: event index; -1: injection chunk
  int32_t pix0, pix1;
  int32_t slot;      // row of the partial-result buffer
  int64_t s0, s1;    // sample (or injection) range
};

// A pixel split over several consecutive slots; merged and gated before combine.
struct SplitPix {
  int32_t slot0, n_parts;
};

// Packed sample (the sweep's input record), precision T.
template <typename T>
struct Samp {
  T m1d, m2d;      // detector-frame masses
  T lm1d, lm2d;    // log2 of them
  T dlc;           // d_L / c  [Mpc s/km]
  T nlp;           // -ln(prior) / ln 2
  T lq;            // log2(m2d / m1d)
  T dlc_lo;        // d_L / c - dlc (rounding residual; 0 in FP64)
};

// Fields of one partial result (per work item and Lambda).
constexpr int NF_FWD = 4;              // R, S1, S2, n_pass
constexpr int NF_GRAD = 4 + 16;        // + sum w * dln w / dLambda

struct SweepArgs {
  const void* samp;          // Samp<T>[n_samp]
  const void* inj;           // Samp<T>[n_inj]
  const int64_t* pix_off;    // [n_pix + 1]
  const int32_t* pix_row;    // [n_pix]
  const void* los;           // [rows][n_z] of T
  const void* sky;           // [n_z] of T
  int32_t n_z;
  double z_max;
  const double* unode;       // [B][n_z] FP64 U(z_k) = (1+z_k) I(z_k) at the table nodes (FP32 adjoint), or null
  const WorkItem* items;     // in slot order
  const int32_t* order;      // processing order of items
  int32_t* item_ctr;         // [B] per-tile counters of handed-out items (zeroed by setup), or
                             // null: items dealt to wavefronts by a fixed stride
  int32_t n_items;
  const void* lamc;          // LamC<T>[B]
  const void* cos_tab;       // [B][NU+1] of T2
  const void* win_tab;       // [B][NW+1] of T2
  const void* win_grad_tab;  // [B][N_WIN_GRAD][NWG+1] of T2 (adjoint only)
  int32_t B;
  double neff_min;
  int32_t gate_mode;
  int32_t z_prior;           // 0: LOS tables; 1: comoving volume (spectral sirens)
  int32_t skip_events;       // 1: only the injection items (the KDE numerator sweeps events itself)
  double* part;              // [B][n_items][NF]
};

// KDE numerator: per (pixel, point) record {R, T, S1, S2}, every sum scaled by
// 2^-R; T = integral of KDE x redshift prior x rate over the pixel's grid (0
// when the pixel fails the gate), S1/S2 the Eq. (8) sums of its weights.
constexpr int NF_KDE = 4;
// Largest redshift grid of the KDE numerator.
constexpr int KDE_GRID_MAX = 1024;
// Pixels with more samples than this are split into parts of this many
// samples for the KDE's grid stage (one wavefront task per part).
constexpr int KDE_PART = 256;

// One part of a pixel for the KDE numerator: samples [lo, hi) of the pixel
// (local indices) in the grid stage; part 0 of a pixel has lo = 0.
struct KdePart {
  int64_t pix;
  int32_t lo, hi;
};

struct KdeArgs {
  const void* samp;          // Samp<T>[n_samp]
  const int64_t* pix_off;    // [n_pix + 1]
  const int32_t* pix_row;    // [n_pix]
  const int32_t* perm;       // [n_samp] per pixel: local indices in ascending d_L order
  const void* los;           // [rows][n_z] of T
  int32_t n_z;
  double z_max;
  int64_t n_pix;
  const int32_t* order;      // [n_pix] pixels by decreasing sample count (batched kernel), or null
  const KdePart* parts;      // [n_parts], pixel-major; null: one part per pixel (n_parts = n_pix)
  int64_t n_parts;
  const void* lamc;          // LamC<T>[B]
  const void* cos_tab;       // [B][NU+1] of T2
  const void* win_tab;       // [B][NW+1] of T2
  int32_t B;
  int32_t bandwidth;         // 0 Scott, 1 Silverman, 2 biweight
  int32_t n_grid;            // grid nodes (2 ... KDE_GRID_MAX)
  double tau;                // grid margin in bandwidths
  double neff_min;
  int32_t gate_mode;
  double* out;               // [B][n_parts][NF_KDE]: {R, T, S1, S2}; S1, S2 only on part 0
  unsigned long long* evals; // [0] (sample, node) kernel terms, [1] grid nodes of the launch (zeroed before it)
  int32_t* pix_ctr;          // [B] per-tile counters of handed-out pixel batches (batched kernel;
                             // zeroed by setup), or null: pixels dealt by a fixed stride
};
// Pixels the batched KDE kernel takes per counter increment.
constexpr int KDE_PIX_BATCH = 16;

struct GateSplitArgs {
  double* part;              // [B][n_items][nf]
  int32_t n_items;
  int32_t nf;
  int32_t B;
  const SplitPix* splits;
  int32_t n_split;
  double neff_min;
  int32_t gate_mode;
};

// Combine slice record: sum of ln L_i, events used, flags, selection (R, S1,
// S2), 16 event basis sums, 16 selection basis sums.
constexpr int NF_CSLICE = 38;

struct CombineArgs {
  const double* part;        // [B][n_items][nf]
  int32_t n_items;
  int32_t nf;                // NF_FWD or NF_GRAD
  int32_t B;
  int32_t n_events;
  const int32_t* ev_item_off;   // [n_events + 1] slot ranges
  int32_t inj_slot0, inj_slot1;
  const double* ln_ns;          // [n_events] ln N_s,i
  double ln_ndraw;
  double neff_min;
  int32_t gate_mode;
  const int* valid;             // [B] (from setup)
  double* logL;                 // [B]
  double* logL_event;           // [B][n_events] or null
  double* neff_event;           // [B][n_events] or null
  double* neff_sel;             // [B] or null
  uint32_t* flags;              // [B] or null
  double* grad;                 // [B][16] or null
  const double* gmap;           // [B][N_GMAP] (adjoint only)
  const double* kde;            // [B][n_events][NF_KDE] event records (KDE numerator) or null
  int32_t wave_events;          // 1: one wavefront merges an event's items (events of many items)
  int32_t n_slices;             // workgroups per point (events and injection slots strided over them)
  double* cpart;                // [B][n_slices][NF_CSLICE] slice records when n_slices > 1
  int32_t* slice_ctr;           // [B] finished slices per point (zeroed by setup): the last one merges
                                // the slice records (small grids); null: a launch of its own does
};

}  // namespace dsl
