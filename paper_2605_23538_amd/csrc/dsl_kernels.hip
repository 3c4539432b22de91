// HIP kernels (gfx950) of the dark-siren population log-likelihood.
//
//   setup_kernel    two workgroups per hyperparameter point: FP64 cosmology and
//                   mass-model constants, the z(d_L) inverse table and the
//                   smoothing-window tables (Eq. 1 and the MultiPeak model).
//   sweep_kernel    persistent sweep over work items (runs of whole pixels of
//                   one event, or runs of injections): per-sample weights of
//                   Eq. (7), FP64 per-pixel sums, the Eq. (8) gate, per-item
//                   partial sums; optionally the adjoint (d ln w / d Lambda).
//   combine_kernel  one workgroup per point: per-event ln L_i, N_eff,i, the
//                   selection term and ln L (Eqs. 3-5), in a fixed order.
//
// Weights are carried as w = 2^n * lin (integer n, FP32 or FP64 lin) so every
// factor that can over- or underflow (prior, power laws, smoothing tails) is
// added into the binary exponent, and FP64 sums are rescaled by exact powers
// of two: the log-sum-exp needs no transcendental per merge.
#include "dsl_device.h"

namespace dsl {

// ---------------------------------------------------------------------------
// FP64 helpers of the setup kernel
// ---------------------------------------------------------------------------
__device__ inline double E_of(double z, double Om) {
  const double x = 1.0 + z;
  return sqrt(Om * x * x * x + (1.0 - Om));
}

// 8-point Gauss-Legendre nodes/weights on [-1, 1].
__constant__ double GL8_X[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                                -0.1834346424956498, 0.1834346424956498, 0.5255324099163290,
                                0.7966664774136267, 0.9602898564975363};
__constant__ double GL8_W[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                                0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                                0.2223810344533745, 0.1012285362903763};

// Smoothing window S(m) and its logarithmic derivatives (x = m - m_min).
struct SmoothD {
  double S, omS;   // S and 1 - S
  double dlnS_dm, dlnS_ddm;
};
__device__ inline SmoothD smooth_d(double x, double dm) {
  SmoothD r;
  if (x <= 0.0) { r.S = 0.0; r.omS = 1.0; r.dlnS_dm = 0.0; r.dlnS_ddm = 0.0; return r; }
  if (x >= dm) { r.S = 1.0; r.omS = 0.0; r.dlnS_dm = 0.0; r.dlnS_ddm = 0.0; return r; }
  const double y = dm / x + dm / (x - dm);
  if (y > 0) { const double e = exp(-y); r.S = e / (1.0 + e); r.omS = 1.0 / (1.0 + e); }
  else { const double e = exp(y); r.S = 1.0 / (1.0 + e); r.omS = e / (1.0 + e); }
  const double dy_dm = -dm / (x * x) - dm / ((x - dm) * (x - dm));
  const double dy_ddm = 1.0 / x + x / ((x - dm) * (x - dm));
  r.dlnS_dm = -r.omS * dy_dm;
  r.dlnS_ddm = -r.omS * dy_ddm;
  return r;
}

__device__ inline double log_dPhi(double mu, double sig, double lo, double hi) {
  // ln(Phi((hi-mu)/sig) - Phi((lo-mu)/sig)), stable in both tails.
  const double a = (lo - mu) / sig, b = (hi - mu) / sig;
  const double r2 = 0.70710678118654752440;
  double d;
  if (a > 0) d = 0.5 * (erfc(a * r2) - erfc(b * r2));
  else if (b < 0) d = 0.5 * (erfc(-b * r2) - erfc(-a * r2));
  else d = 1.0 - 0.5 * erfc(-a * r2) - 0.5 * erfc(b * r2);
  return log(d);
}

// In-place inclusive scan of n_seg segments of n entries each, x[seg * n + i],
// by the whole workgroup (Hillis-Steele: a fixed shape, so the sums do not
// depend on timing).  tmp holds n_seg * n entries.
__device__ void block_scan(double* x, int n, int n_seg, double* tmp) {
  const int tot = n * n_seg;
  for (int off = 1; off < n; off <<= 1) {
    for (int i = threadIdx.x; i < tot; i += blockDim.x) tmp[i] = (i % n) >= off ? x[i - off] : 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < tot; i += blockDim.x) x[i] += tmp[i];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// setup: per-Lambda constants and tables (FP64), two workgroups per point
// ---------------------------------------------------------------------------
constexpr int SETUP_THREADS = 1024;
template <typename T>
__global__ __launch_bounds__(SETUP_THREADS) void setup_kernel(const double* __restrict__ lam, int B, double z_max,
                                                    LamC<T>* __restrict__ lamc,
                                                    typename V2<T>::t* __restrict__ cos_tab,
                                                    typename V2<T>::t* __restrict__ win_tab,
                                                    typename V2<T>::t* __restrict__ win_grad_tab,
                                                    int* __restrict__ valid_out, double* __restrict__ gmap,
                                                    double* __restrict__ unode, int n_z,
                                                    int32_t* __restrict__ item_ctr) {
  using T2 = typename V2<T>::t;
  constexpr int NU = Tab<T>::NU, NW = Tab<T>::NW, NWG = Tab<T>::NWG;
  const int b = blockIdx.x;
  if (b >= B) return;
  const double* L = lam + 16 * b;
  const double H0 = L[0], Om = L[1], alpha = L[2], beta = L[3], mmin = L[4], mmax = L[5], dm = L[6];
  const double muL = L[7], sL = L[8], muH = L[9], sH = L[10], lg = L[11], ll = L[12];
  const double gam = L[13], kap = L[14], zp = L[15];
  bool ok = true;
  for (int i = 0; i < 16; ++i) ok = ok && isfinite(L[i]);
  ok = ok && H0 > 0 && Om >= 0 && Om <= 1 && mmin > 0 && mmin < mmax && dm >= 0 && sL > 0 && sH > 0 &&
       lg >= 0 && lg <= 1 && ll >= 0 && ll <= 1 && zp > -1;
  __shared__ double zw_s[4];
  __shared__ double cum[NW + 1];
  __shared__ double cumg[3][NW + 1];
  const int tid = threadIdx.x;
  const double M = mmin + dm;
  const double s = beta + 1.0;

  // two workgroups per point: part 0 the cosmology and rate, part 1 the mass model
  const int part = blockIdx.y;
  LamC<T>& c = lamc[b];
  // (the sweep's and the KDE kernel's tiles number at most B each; then the
  // combine's per-point slice counters)
  if (item_ctr && part == 0 && tid == 0) item_ctr[b] = item_ctr[B + b] = item_ctr[2 * B + b] = 0;
  if (part == 0) {
    // --- I(z) on KZ uniform panels (8-point Gauss-Legendre each), prefix-summed.
    constexpr int KZ = KZ_I;
    __shared__ double Itab[KZ + 1];
    const double hz = z_max / KZ;
    for (int k = tid; k < KZ; k += blockDim.x) {
      double sacc = 0.0;
      if (ok) {
        const double c = (k + 0.5) * hz;
        for (int q = 0; q < 8; ++q) sacc += GL8_W[q] / E_of(c + 0.5 * hz * GL8_X[q], Om);
        sacc *= 0.5 * hz;
      }
      Itab[k + 1] = sacc;
    }
    __shared__ double scan_tmp[KZ];
    if (tid == 0) Itab[0] = 0.0;
    __syncthreads();
    block_scan(Itab + 1, KZ, 1, scan_tmp);
    // I(z) = Itab[k] + 8-point Gauss-Legendre over [z_k, z]
    auto I_at = [&](double z) {
      int k = (int)(z / hz);
      k = k < 0 ? 0 : (k > KZ - 1 ? KZ - 1 : k);
      const double a = k * hz, h = z - a;
      double sacc = 0.0;
      for (int q = 0; q < 8; ++q) sacc += GL8_W[q] / E_of(a + 0.5 * h * (GL8_X[q] + 1.0), Om);
      return Itab[k] + 0.5 * h * sacc;
    };
    if (unode) {   // U(z_k) = (1+z_k) I(z_k) at the redshift-table nodes (FP32 adjoint)
      const double dzn = z_max / (double)(n_z - 1);
      for (int k = tid; k < n_z; k += blockDim.x) {
        const double zk = k * dzn;
        unode[(size_t)b * n_z + k] = ok ? (1.0 + zk) * I_at(zk) : 0.0;
      }
    }
    // --- inverse distance table: y(v) = z/u at v_k = 1 + k h_v, u = (v^2-1)/4.
    const double umax = ok ? (1.0 + z_max) * Itab[KZ] : 1.0;
    const double vmax = sqrt(1.0 + 4.0 * umax);
    const double hv = (vmax - 1.0) / NU;
    for (int k = tid; k <= NU; k += blockDim.x) {
      double y = 1.0, dy = -(1.0 - 0.75 * Om) * 0.5;  // limits at u = 0
      if (k > 0 && ok) {
        const double dv = k * hv;
        const double u = dv * (2.0 + dv) * 0.25;
        const double v = 1.0 + dv;
        // bracket: the panel [z_j, z_j+1] with D(z_j) <= u <= D(z_j+1), D = (1+z) I
        int lo = 0, hi = KZ;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if ((1.0 + mid * hz) * Itab[mid] <= u) lo = mid; else hi = mid;
        }
        const double za = lo * hz, zb = hi * hz;
        const double Da = (1.0 + za) * Itab[lo], Db = (1.0 + zb) * Itab[hi];
        double z = za + (zb - za) * (u - Da) / (Db - Da);
        for (int it = 0; it < 12; ++it) {
          const double I = I_at(z);
          const double f = (1.0 + z) * I - u;
          double zn = z - f / (I + (1.0 + z) / E_of(z, Om));
          zn = fmin(fmax(zn, za), zb);
          const bool done = fabs(zn - z) <= 4e-16 * zn;
          z = zn;
          if (done) break;
        }
        const double I = I_at(z);
        const double zp_u = 1.0 / (I + (1.0 + z) / E_of(z, Om));
        y = z / u;
        dy = (zp_u * u - z) / (u * u) * (0.5 * v);
      }
      T2 e;
      e.x = (T)y;
      e.y = (T)(dy * hv);
      cos_tab[(size_t)b * (NU + 1) + k] = e;
    }

    if (tid == 0) {
      c.H0 = (T)H0;
      c.H0_lo = (T)(H0 - (double)(T)H0);
      c.u_max = (T)umax;
      c.inv_hv = (T)(1.0 / hv);
      c.Om = (T)Om;
      c.OL = (T)(1.0 - Om);
      c.c0 = (T)log2(H0 / C_KMS);
      c.gm3 = (T)(gam - 3.0);
      c.gk = (T)(gam + kap);
      c.Lp = (T)log2(1.0 + zp);
      c.gamma = (T)gam;
      c.kappa = (T)kap;
      c.inv_opzp = (T)(1.0 / (1.0 + zp));
      c.inv_H0 = (T)(1.0 / H0);
      c.om_case = Om < 1e-6 ? 1 : (Om > 1 - 1e-6 ? 2 : 0);
      c.k23 = c.om_case == 0 ? (T)((2.0 / 3.0) / (1.0 - Om)) : (T)0;
      c.hOm = c.om_case == 0 ? (T)(0.5 / Om) : (T)0;
      c.valid = ok ? 1 : 0;
      valid_out[b] = ok ? 1 : 0;
      if (gmap) {
        double* gm = gmap + (size_t)b * N_GMAP;
        gm[0] = 1.0 / H0;
        gm[20] = (gam + kap) / (1.0 + zp);
        gm[21] = LN2;
        gm[22] = 0.0;
        gm[23] = 0.0;
      }
    }
    return;
  }
  // --- truncated-Gaussian normalisers of the two peaks and their derivatives
  // (-ln dPhi with respect to mu, sigma, m_min, m_max): one lane each, in the
  // last wavefront, beside the window integrals.
  __shared__ double gpk[2][5];
  const int gl = tid - ((int)blockDim.x - 2);
  if (gl >= 0) {
    const double r2pi = 2.5066282746310002;
    const double mu = gl == 0 ? muL : muH, sg = gl == 0 ? sL : sH;
    const double ldP = ok ? log_dPhi(mu, sg, mmin, mmax) : 0.0;
    const double dP = exp(ldP);
    const double za = (mmin - mu) / sg, zb = (mmax - mu) / sg;
    const double pa = exp(-0.5 * za * za) / r2pi, pb = exp(-0.5 * zb * zb) / r2pi;
    gpk[gl][0] = -log(sg * r2pi) - ldP;
    gpk[gl][1] = -(-pb + pa) / sg / dP;
    gpk[gl][2] = -1.0 / sg - (-pb * zb + pa * za) / sg / dP;
    gpk[gl][3] = pa / sg / dP;
    gpk[gl][4] = -pb / sg / dP;
  }
  // --- smoothing-window integrals on NW panels (Gauss-Legendre 8 x 2 per
  // panel), one quarter panel (four nodes) per thread: Z = int m^beta S and,
  // for the adjoint, int m^beta ln(m) S, J = int m^beta S' and K = int m^beta
  // tau S' (S' = dS/dm, tau = (m - m_min) / dm).  S(m) depends on m_min and dm
  // only through tau, so dS/dm_min = -S' and dS/d(dm) = -tau S'.
  __shared__ double qsum[4][4 * NW];
  const bool win = ok && dm > 0;
  for (int i = tid; i < 4 * NW; i += blockDim.x) {
    const int j = i >> 2, qtr = i & 3;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    if (win) {
      const double ta = (double)j / NW, h = 1.0 / NW;
      const double c = ta + ((qtr >> 1) + 0.5) * 0.5 * h;
      for (int u = 0; u < 4; ++u) {
        const int q = 4 * (qtr & 1) + u;
        const double t = c + 0.25 * h * GL8_X[q];
        const double m = mmin + dm * t;
        const SmoothD sd = smooth_d(m - mmin, dm);
        const double wq = GL8_W[q] * 0.25 * h * dm;
        const double lm = log(m);
        const double mb = exp(beta * lm);
        a0 += wq * mb * sd.S;
        a1 += wq * mb * lm * sd.S;
        a2 += wq * mb * sd.S * sd.dlnS_dm;
        a3 += wq * mb * sd.S * sd.dlnS_dm * t;
      }
    }
    qsum[0][i] = a0;
    qsum[1][i] = a1;
    qsum[2][i] = a2;
    qsum[3][i] = a3;
  }
  __syncthreads();
  // running sums over the panels of the four arrays (each panel's quarters
  // summed in order, then a block scan)
  __shared__ double pan[4 * NW], pan_tmp[4 * NW];
  for (int i = tid; i < 4 * NW; i += blockDim.x) {
    const double* src = qsum[i / NW] + 4 * (i % NW);
    pan[i] = (src[0] + src[1]) + (src[2] + src[3]);
  }
  __syncthreads();
  block_scan(pan, NW, 4, pan_tmp);
  for (int i = tid; i < 4 * (NW + 1); i += blockDim.x) {
    const int a = i / (NW + 1), j = i % (NW + 1);
    double* dst = a == 0 ? cum : cumg[a - 1];
    dst[j] = j == 0 ? 0.0 : pan[a * NW + j - 1];
  }
  if (tid < 4) {
    const double run = pan[tid * NW + NW - 1];
    // With delta_m = 0 the window integrals vanish, but two of their derivatives
    // do not: the window integral of m^beta S is m_min^beta delta_m / 2 to first
    // order (the window's mean over its width is 1/2), and the step at m_min
    // moves with m_min.  Divided by M^s = m_min^(beta+1), the one-sided limits
    // are d/d m_min -> -1/m_min and d/d delta_m -> -1/(2 m_min).
    const double zw0 = (ok && dm == 0.0) ? (tid == 2 ? -1.0 / mmin : (tid == 3 ? -0.5 / mmin : 0.0)) : 0.0;
    // window integrals of m^beta dS/d(m_min) = -J and of m^beta dS/d(dm) = -K
    const double sgn = tid >= 2 ? -1.0 : 1.0;
    zw_s[tid] = win ? sgn * run / exp(s * log(M)) : zw0;
  }
  __syncthreads();
  // rho(t) = Z / (S m^s) and its t-derivative (Hermite data), t = (m - m_min) / dm.
  for (int j = tid; j <= NW; j += blockDim.x) {
    double rho = 0, drho = 0;
    if (win && j > 0) {
      const double t = (double)j / NW;
      const double m = mmin + dm * t;
      const SmoothD sd = smooth_d(m - mmin, dm);
      const double ms = exp(s * log(m));
      const double Sd = (j == NW) ? 1.0 : sd.S;
      rho = cum[j] / (Sd * ms);
      const double dlnS = (j == NW) ? 0.0 : sd.dlnS_dm;
      drho = dm * (1.0 / m - rho * (dlnS + s / m));
    }
    T2 e;
    e.x = (T)rho;
    e.y = (T)(drho / NW);
    win_tab[(size_t)b * (NW + 1) + j] = e;
  }
  // Adjoint tables on every second node: the window-integral parts of the
  // derivatives of rho at fixed m1,
  //   d rho/d beta  = D,                D = int m^beta ln(m/m1) S dm / (S m1^s),
  //   d rho/d m_min = -J~ + rho S'/S,   J~ = J / (S m1^s),
  //   d rho/d dm    = -K~ + rho t S'/S, K~ = K / (S m1^s),
  // whose local parts (S'/S at m1) the sweep adds per sample.  Tangents are
  // analytic: d/dt [I(t) / (S m1^s)] = dm (f(m1) / (S m1^s) - [I / (S m1^s)] (S'/S + s/m1))
  // for an integral I of integrand f (for D also the -dm rho/m1 of ln(m/m1)).
  if (win_grad_tab) {
    for (int i = tid; i < 3 * (NWG + 1); i += blockDim.x) {
      const int q = i / (NWG + 1), jc = i % (NWG + 1), j = (NW / NWG) * jc;
      double v = 0.0, d = 0.0;
      if (win && j > 0) {
        const double t = (double)j / NW;
        const double m = mmin + dm * t;
        const SmoothD sd = smooth_d(m - mmin, dm);
        const double den = ((j == NW) ? 1.0 : sd.S) * exp(s * log(m));
        const double dl = (j == NW) ? 0.0 : sd.dlnS_dm;
        const double g = dl + s / m;
        if (q == 0) {
          const double rho = cum[j] / den;
          v = (cumg[0][j] - log(m) * cum[j]) / den;
          d = -dm * (rho / m + v * g);
        } else if (q == 1) {
          v = cumg[1][j] / den;
          d = dm * (dl / m - v * g);
        } else {
          v = cumg[2][j] / den;
          d = dm * (t * dl / m - v * g);
        }
      }
      T2 e;
      e.x = (T)v;
      e.y = (T)(d / NWG);
      win_grad_tab[((size_t)b * 3 + q) * (NWG + 1) + jc] = e;
    }
  }

  if (tid == 0) {
    double lnbP, dbPa, dbPmin, dbPmax;
    if (fabs(alpha - 1.0) < 1e-10) {
      const double lr = log(mmax / mmin);
      lnbP = -log(lr);
      dbPa = 0.5 * (log(mmax) + log(mmin));     // limit of the alpha derivative at alpha = 1
      dbPmin = 1.0 / (mmin * lr);
      dbPmax = -1.0 / (mmax * lr);
    } else {
      const double a1 = 1.0 - alpha;
      const double A = exp(a1 * log(mmax)), Bm = exp(a1 * log(mmin));
      lnbP = log(fabs(a1)) - log(fabs(A - Bm));
      // d/d alpha of ln|1-alpha| - ln|A - B|, with dA/dalpha = -A ln mmax
      dbPa = -1.0 / a1 + (A * log(mmax) - Bm * log(mmin)) / (A - Bm);
      dbPmin = a1 * Bm / mmin / (A - Bm);
      dbPmax = -a1 * A / mmax / (A - Bm);
    }
    const double lnbL = gpk[0][0], lnbH = gpk[1][0];
    const double dLmu = gpk[0][1], dLsg = gpk[0][2], dLlo = gpk[0][3], dLhi = gpk[0][4];
    const double dHmu = gpk[1][1], dHsg = gpk[1][2], dHlo = gpk[1][3], dHhi = gpk[1][4];
    const double l2 = LOG2E;
    c.alpha = (T)alpha;
    c.beta = (T)beta;
    c.mmin = (T)mmin;
    c.mmin_lo = (T)(mmin - (double)(T)mmin);
    c.mmax = (T)mmax;
    c.dm = (T)dm;
    c.inv_dm = dm > 0 ? (T)(1.0 / dm) : (T)0;
    c.cP = (T)((lg < 1 ? log(1.0 - lg) : -INFINITY) * l2 + lnbP * l2);
    c.cL = (T)((lg * ll > 0 ? log(lg * ll) : -INFINITY) * l2 + lnbL * l2);
    c.cH = (T)((lg * (1 - ll) > 0 ? log(lg * (1 - ll)) : -INFINITY) * l2 + lnbH * l2);
    c.muL = (T)muL;
    c.muL_lo = (T)(muL - (double)(T)muL);
    c.kL = (T)(-l2 / (2 * sL * sL));
    c.muH = (T)muH;
    c.muH_lo = (T)(muH - (double)(T)muH);
    c.kH = (T)(-l2 / (2 * sH * sH));
    c.s = (T)s;
    c.inv_s = (T)(1.0 / s);
    c.lM = (T)log2(M);
    c.inv_M = (T)(1.0 / M);
    c.zw = (T)zw_s[0];
    c.dbP_alpha = (T)dbPa;
    c.dbP_mmin = (T)dbPmin;
    c.dbP_mmax = (T)dbPmax;
    c.dbL_mu = (T)dLmu;
    c.dbL_sig = (T)dLsg;
    c.dbL_mmin = (T)dLlo;
    c.dbL_mmax = (T)dLhi;
    c.dbH_mu = (T)dHmu;
    c.dbH_sig = (T)dHsg;
    c.dbH_mmin = (T)dHlo;
    c.dbH_mmax = (T)dHhi;
    c.sigL = (T)sL;
    c.sigH = (T)sH;
    c.lg = (T)lg;
    c.ll = (T)ll;
    c.zw_beta = (T)zw_s[1];
    c.zw_mmin = (T)zw_s[2];
    c.zw_dm = (T)zw_s[3];
    c.isL2 = (T)(1.0 / (sL * sL));
    c.isL3 = (T)(1.0 / (sL * sL * sL));
    c.isH2 = (T)(1.0 / (sH * sH));
    c.isH3 = (T)(1.0 / (sH * sH * sH));
    c.aPg = lg < 1 ? (T)(1.0 / (1.0 - lg)) : (T)0;
    c.aLg = lg > 0 ? (T)(1.0 / lg) : (T)0;
    c.aLl = ll > 0 ? (T)(1.0 / ll) : (T)0;
    c.aHl = ll < 1 ? (T)(1.0 / (1.0 - ll)) : (T)0;
    c.inv_s2 = (T)(1.0 / (s * s));
    if (gmap) {
      double* gm = gmap + (size_t)b * N_GMAP;
      gm[1] = dbPa;
      gm[2] = dbPmin;
      gm[3] = dLlo;
      gm[4] = dHlo;
      gm[5] = dbPmax;
      gm[6] = dLhi;
      gm[7] = dHhi;
      gm[8] = dLmu;
      gm[9] = dLsg;
      gm[10] = dHmu;
      gm[11] = dHsg;
      gm[12] = 1.0 / (sL * sL);
      gm[13] = 1.0 / (sL * sL * sL);
      gm[14] = 1.0 / (sH * sH);
      gm[15] = 1.0 / (sH * sH * sH);
      gm[16] = lg < 1 ? 1.0 / (1.0 - lg) : 0.0;
      gm[17] = lg > 0 ? 1.0 / lg : 0.0;
      gm[18] = ll > 0 ? 1.0 / ll : 0.0;
      gm[19] = ll < 1 ? 1.0 / (1.0 - ll) : 0.0;
    }
  }
}

// Item-level sums: S1, S2 in FP64; the 16 adjoint basis sums in GT (FP32 for
// the FP32 sweep, like the pixel-level ones: an item merges a few pixels).
template <bool GRAD, typename GT = double>
struct ItemAcc {
  int R;
  double S1, S2;
  GT G[GRAD ? 16 : 1];
  __device__ __forceinline__ void zero() {
    R = R_SENTINEL;
    S1 = 0;
    S2 = 0;
#pragma unroll
    for (int p = 0; p < (GRAD ? 16 : 1); ++p) G[p] = 0;
  }
  template <typename BT>
  __device__ __forceinline__ void merge(const PixAcc<GRAD, BT>& o) {
    const int Rm = R > o.R ? R : o.R;
    const int da = R - Rm, db = o.R - Rm;
    S1 = ldexp(S1, da) + ldexp(o.S1, db);
    S2 = ldexp(S2, 2 * da) + ldexp(o.S2, 2 * db);
    if constexpr (GRAD) {
#pragma unroll
      for (int p = 0; p < 16; ++p) G[p] = ldexp(G[p], da) + ldexp((GT)o.G[p], db);
    }
    R = Rm;
  }
};

// One run of samples [s0, s1) accumulated into acc; the next record is
// loaded while the current one is evaluated.  The bounds are the same on
// every lane: as scalars they keep the loop's counter and the record
// addresses off the vector unit.
template <typename T, int GL, bool GRAD, bool SPEC, typename AccT>
__device__ __forceinline__ void sweep_run(const Samp<T>* __restrict__ base, int64_t s0, int64_t s1, int sg,
                                          bool live, const LamC<T>& c, const TabView<T>& tv, int lam,
                                          const T* __restrict__ tab, int n_z, T inv_dz, AccT& acc,
                                          T* g, const double* __restrict__ unode) {
  constexpr int NS = 64 / GL;
  s0 = uniform64(s0);
  s1 = uniform64(s1);
  if (s1 <= s0) return;
  if constexpr (NS == 1) {
    // one sample per wavefront (a 32-bit count from the run's first record:
    // the scalar unit has no signed 64-bit compare)
    const Samp<T>* __restrict__ rp = base + s0;
    const int n = (int)(s1 - s0);
    Samp<T> nxt = ld_samp<T, 1>(rp, 0);
    for (int k = 0; k < n; ++k) {
      const Samp<T> cur = nxt;
      if (k + 1 < n) nxt = ld_samp<T, 1>(rp, k + 1);
      if (live) {
        int nw;
        T lin;
        eval_weight<T, GL, GRAD, false, SPEC>(cur, c, tv, lam, tab, n_z, inv_dz, nw, lin, g, nullptr, unode);
        acc.template add<T>(nw, lin, g);
      }
    }
    return;
  }
  // indices are clamped into the run; with several samples per wavefront two
  // records are in flight (one point per lane leaves little work to hide a load)
  auto at = [&](int64_t sb) { const int64_t i = sb + sg; return i < s1 ? i : s1 - 1; };
  Samp<T> nxt = ld_samp<T, NS>(base, at(s0));
  Samp<T> nxt2 = ld_samp<T, NS>(base, at(s0 + NS));
  for (int64_t sb = s0; sb < s1; sb += NS) {
    const Samp<T> cur = nxt;
    nxt = nxt2;
    if (sb + 2 * NS < s1) nxt2 = ld_samp<T, NS>(base, at(sb + 2 * NS));
    if (sb + sg < s1 && live) {
      int n;
      T lin;
      eval_weight<T, GL, GRAD, false, SPEC>(cur, c, tv, lam, tab, n_z, inv_dz, n, lin, g, nullptr, unode);
      acc.template add<T>(n, lin, g);
    }
  }
}

// ---------------------------------------------------------------------------
// sweep
// ---------------------------------------------------------------------------
// Largest workgroup of a sweep variant: 768 threads (12 wavefronts, 3 per SIMD
// at <= 168 VGPRs) for the FP32 adjoint -- the 64-point tables take 117 KB of
// LDS, so one workgroup per CU -- and 512 otherwise.
template <typename T, int GL, bool GRAD>
struct SweepMaxThreads { static constexpr int N = (sizeof(T) == 4 && GRAD) ? 768 : 512; };

template <typename T, int GL, bool GRAD, bool SPEC>
__global__ __attribute__((amdgpu_flat_work_group_size(1, SweepMaxThreads<T, GL, GRAD>::N))) void sweep_kernel(
    SweepArgs a) {
  using T2 = typename V2<T>::t;
  constexpr int NU = Tab<T>::NU, NW = Tab<T>::NW;
  constexpr int NF = GRAD ? NF_GRAD : NF_FWD;
  extern __shared__ __align__(16) unsigned char smem[];
  T2* cosL = reinterpret_cast<T2*>(smem);
  T2* winL = cosL + (NU + 1) * GL;
  T2* wgL = winL + (NW + 1) * GL;
  const int tile = blockIdx.y;
  const int tid = threadIdx.x;
  const T2* cos_g = reinterpret_cast<const T2*>(a.cos_tab);
  const T2* win_g = reinterpret_cast<const T2*>(a.win_tab);
  const T2* wg_g = reinterpret_cast<const T2*>(a.win_grad_tab);
  for (int i = tid; i < (NU + 1) * GL; i += blockDim.x) {
    const int k = i / GL, l = i % GL, b = tile * GL + l;
    cosL[i] = b < a.B ? cos_g[(size_t)b * (NU + 1) + k] : T2{};
  }
  for (int i = tid; i < (NW + 1) * GL; i += blockDim.x) {
    const int k = i / GL, l = i % GL, b = tile * GL + l;
    winL[i] = b < a.B ? win_g[(size_t)b * (NW + 1) + k] : T2{};
  }
  if constexpr (GRAD) {
    constexpr int NWG = Tab<T>::NWG;
    for (int i = tid; i < 3 * (NWG + 1) * GL; i += blockDim.x) {
      const int q = i / ((NWG + 1) * GL), rem = i % ((NWG + 1) * GL);
      const int k = rem / GL, l = rem % GL, b = tile * GL + l;
      wgL[i] = b < a.B ? wg_g[((size_t)b * 3 + q) * (NWG + 1) + k] : T2{};
    }
  }
  __syncthreads();
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: item bounds stay scalar
  const int nwaves = blockDim.x >> 6;
  const int lam = lane % GL;
  const int sg = lane / GL;
  const int b = tile * GL + lam;
  const bool active = b < a.B;
  const LamC<T>* lamc = reinterpret_cast<const LamC<T>*>(a.lamc);
  const LamC<T> c = lamc[active ? b : 0];
  const bool live = active && c.valid;
  const TabView<T> tv{cosL, winL, wgL};
  const Samp<T>* __restrict__ samp = reinterpret_cast<const Samp<T>*>(a.samp);
  const Samp<T>* __restrict__ inj = reinterpret_cast<const Samp<T>*>(a.inj);
  const T inv_dz = (T)((a.n_z - 1) / a.z_max);
  const T* __restrict__ los = reinterpret_cast<const T*>(a.los);
  const T* __restrict__ sky = reinterpret_cast<const T*>(a.sky);
  // the point's FP64 node values (FP32 table prior only): cells of samples near table nodes
  const double* __restrict__ un = (a.unode && !SPEC && active) ? a.unode + (size_t)b * a.n_z : nullptr;
  T g[GRAD ? 16 : 1];

  // Work items: each wavefront's first by a fixed stride, the rest from the
  // tile's counter (the list runs largest first, so a fixed stride would give
  // the same workgroups the largest item of every round); every item writes
  // its own slot, so the results do not depend on which wavefront took it.
  // (a list the first round covers needs no counter)
  const int n_first = gridDim.x * nwaves;
  int32_t* const ctr = a.item_ctr && a.n_items > n_first ? a.item_ctr + tile : nullptr;
  auto next_item = [&](int it) -> int {
    if (!ctr) return it + n_first;
    int v = 0;
    if (lane == 0) v = atomicAdd(ctr, 1);
    return n_first + __builtin_amdgcn_readfirstlane(v);
  };
  for (int it = blockIdx.x * nwaves + wave; it < a.n_items; it = next_item(it)) {
    const WorkItem w = a.items[a.order[it]];
    if (a.skip_events && w.event >= 0) continue;
    ItemAcc<GRAD, T> chunk;
    chunk.zero();
    int npass = 0;
    if (w.event >= 0 && w.pix1 == w.pix0) {
      // part of a large pixel: ungated sums, gated after the sweep (gate_split_kernel)
      const T* __restrict__ tab = SPEC ? nullptr : los + (size_t)a.pix_row[w.pix0] * a.n_z;
      PixAcc<GRAD, T> pix;
      pix.zero();
      sweep_run<T, GL, GRAD, SPEC>(samp, w.s0, w.s1, sg, live, c, tv, lam, tab, a.n_z, inv_dz, pix, g, un);
#pragma unroll
      for (int off = GL; off < 64; off <<= 1) pix.xor_merge(off);
      chunk.merge(pix);
    } else if (w.event >= 0) {
      for (int p = w.pix0; p < w.pix1; ++p) {
        const int64_t s0 = a.pix_off[p], s1 = a.pix_off[p + 1];
        const T* __restrict__ tab = SPEC ? nullptr : los + (size_t)a.pix_row[p] * a.n_z;
        PixAcc<GRAD, T> pix;
        pix.zero();
        sweep_run<T, GL, GRAD, SPEC>(samp, s0, s1, sg, live, c, tv, lam, tab, a.n_z, inv_dz, pix, g, un);
#pragma unroll
        for (int off = GL; off < 64; off <<= 1) pix.xor_merge(off);
        bool pass;
        if (a.gate_mode == 2) pass = pix.S1 > 0;
        else pass = pix.S2 > 0 && pix.S1 * pix.S1 >= a.neff_min * pix.S2;
        if (pass) {
          chunk.merge(pix);
          ++npass;
        }
      }
    } else {
      // injections in runs of 256 per lane (the pixel-level sums are FP32 for the adjoint)
      constexpr int64_t VP = 256 * (64 / GL);
      for (int64_t v0 = w.s0; v0 < w.s1; v0 += VP) {
        PixAcc<GRAD, T> pix;
        pix.zero();
        const int64_t v1 = v0 + VP < w.s1 ? v0 + VP : w.s1;
        sweep_run<T, GL, GRAD, SPEC>(inj, v0, v1, sg, live, c, tv, lam, SPEC ? nullptr : sky, a.n_z, inv_dz,
                               pix, g, un);
#pragma unroll
        for (int off = GL; off < 64; off <<= 1) pix.xor_merge(off);
        chunk.merge(pix);
      }
    }
    if (sg == 0 && active) {
      // partial sums laid out [point][item][field]: one lane writes its fields contiguously
      double* out = a.part + ((size_t)b * a.n_items + w.slot) * NF;
      out[0] = (double)chunk.R;
      out[1] = chunk.S1;
      out[2] = chunk.S2;
      out[3] = (double)npass;
      if constexpr (GRAD) {
#pragma unroll
        for (int p = 0; p < 16; ++p) out[4 + p] = chunk.G[p];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// gate of split pixels: one wavefront per (split pixel, point) merges the
// parts (lanes stride over them, then a fixed xor butterfly of exact power-of-
// two rescalings and commutative sums, so every lane holds the same bits),
// applies Eq. (8), writes the result into the first part's slot and clears
// the others.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gate_split_kernel(GateSplitArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= (int64_t)a.n_split * a.B) return;   // whole wavefronts
  const int sp = (int)(w / a.B), b = (int)(w % a.B);
  const SplitPix s = a.splits[sp];
  auto at = [&](int slot, int f) -> double& { return a.part[((size_t)b * a.n_items + slot) * a.nf + f]; };
  const int ng = a.nf - 4;
  double R = -1e300, S1 = 0, S2 = 0;
  double G[16];
  for (int p = 0; p < 16; ++p) G[p] = 0;
  // (R, S1, S2, G) += 2^(r - R) (r, s1, s2, g): rescaled to the larger exponent
  auto merge = [&](double r, double s1, double s2, const double* g) {
    if (!(s1 > 0)) return;
    if (!(S1 > 0)) {
      R = r;
      S1 = s1;
      S2 = s2;
      for (int p = 0; p < ng; ++p) G[p] = g[p];
      return;
    }
    const double Rm = fmax(R, r);
    const int da = (int)(R - Rm), db = (int)(r - Rm);
    S1 = ldexp(S1, da) + ldexp(s1, db);
    S2 = ldexp(S2, 2 * da) + ldexp(s2, 2 * db);
    for (int p = 0; p < ng; ++p) G[p] = ldexp(G[p], da) + ldexp(g[p], db);
    R = Rm;
  };
  for (int k = lane; k < s.n_parts; k += 64) {
    const int sl = s.slot0 + k;
    double g[16];
    for (int p = 0; p < ng; ++p) g[p] = at(sl, 4 + p);
    merge(at(sl, 0), at(sl, 1), at(sl, 2), g);
  }
  for (int off = 1; off < 64; off <<= 1) {
    double g[16];
    for (int p = 0; p < ng; ++p) g[p] = __shfl_xor(G[p], off);
    const double r = __shfl_xor(R, off), s1 = __shfl_xor(S1, off), s2 = __shfl_xor(S2, off);
    merge(r, s1, s2, g);
  }
  bool pass;
  if (a.gate_mode == 2) pass = S1 > 0;
  else pass = S2 > 0 && S1 * S1 >= a.neff_min * S2;
  for (int k = lane; k < s.n_parts; k += 64) {
    const int sl = s.slot0 + k;
    const bool first = k == 0 && pass;
    at(sl, 0) = first ? R : (double)R_SENTINEL;
    at(sl, 1) = first ? S1 : 0.0;
    at(sl, 2) = first ? S2 : 0.0;
    at(sl, 3) = first ? 1.0 : 0.0;
    for (int p = 0; p < ng; ++p) at(sl, 4 + p) = first ? G[p] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// combine: per point, fixed-order reductions
// ---------------------------------------------------------------------------
struct Part3 {
  double R, S1, S2;
};
__device__ inline Part3 pmerge(Part3 x, Part3 y) {
  if (!(x.S1 > 0)) return y;
  if (!(y.S1 > 0)) return x;
  const double Rm = fmax(x.R, y.R);
  Part3 r;
  r.R = Rm;
  r.S1 = ldexp(x.S1, (int)(x.R - Rm)) + ldexp(y.S1, (int)(y.R - Rm));
  r.S2 = ldexp(x.S2, 2 * (int)(x.R - Rm)) + ldexp(y.S2, 2 * (int)(y.R - Rm));
  return r;
}

// ln L, N_eff of the selection term, flags and the gradient map of one point
// from its merged sums (redg / gsel: 16 values with strides rs / gs).
template <bool GRAD>
__device__ void combine_finish(const CombineArgs& a, int b, double acc, double nused, unsigned int flags,
                               const double* redg, int rs, Part3 sel, const double* gsel, int gs) {
  const double ln2 = LN2;
  const bool valid = a.valid[b] != 0;
  {
    const Part3 s = sel;
    unsigned int f = flags;
    double logL = -INFINITY;
    double lna = -INFINITY;
    if (!valid) f |= 1u;
    if (valid && s.S1 > 0) lna = log(s.S1) + s.R * ln2 - a.ln_ndraw;
    else if (valid) f |= 4u;
    if (f == 0) {
      logL = acc - (double)a.n_events * lna;
      if (!isfinite(logL)) {
        f |= 8u;
        logL = -INFINITY;
      }
    }
    a.logL[b] = logL;
    if (a.neff_sel) a.neff_sel[b] = s.S1 > 0 ? s.S1 * s.S1 / s.S2 : 0.0;
    if (a.flags) a.flags[b] = f;
    if constexpr (GRAD) {
      if (a.grad) {
        // basis totals T_j = sum_i B_ij / S1_i - N_det B_sel,j / S1_sel, then the map
        double T[16];
        for (int p = 0; p < 16; ++p) T[p] = (f == 0) ? redg[p * rs] - (double)a.n_events * gsel[p * gs] / s.S1 : 0.0;
        const double* c = a.gmap + (size_t)b * N_GMAP;
        const double T1 = nused - (double)a.n_events;   // coefficient of the constant 1/H0 term
        double g[16];
        g[0] = c[0] * T1 + T[0];
        g[1] = T[1];
        g[2] = c[1] * T[2] - T[3];
        g[3] = T[4];
        g[4] = c[2] * T[2] + c[3] * T[5] + c[4] * T[6] - T[7];
        g[5] = c[5] * T[2] + c[6] * T[5] + c[7] * T[6];
        g[6] = T[8];
        g[7] = c[8] * T[5] + c[12] * T[9];
        g[8] = c[9] * T[5] + c[13] * T[10];
        g[9] = c[10] * T[6] + c[14] * T[11];
        g[10] = c[11] * T[6] + c[15] * T[12];
        g[11] = -c[16] * T[2] + c[17] * (T[5] + T[6]);
        g[12] = c[18] * T[5] - c[19] * T[6];
        g[13] = c[21] * T[13] - T[14];
        g[14] = -T[14];
        g[15] = c[20] * T[15];
        for (int p = 0; p < 16; ++p) a.grad[(size_t)b * 16 + p] = (f == 0) ? g[p] : 0.0;
      }
    }
  }
}

// Merge of one event's item records by one wavefront (lanes stride over the
// items, then a fixed xor butterfly whose merges are exact power-of-two
// rescalings and commutative sums, so every lane ends with the same bits):
// the event's (R, S1, S2) and, with GRAD, its 16 basis sums scaled by 2^R.
// Used when events span many items, where one thread per event would walk
// them serially.
template <bool GRAD>
__device__ __forceinline__ Part3 wave_merge_event(const CombineArgs& a, int b, int e, int lane, double* G) {
  const double* P = a.part + (size_t)b * a.n_items * a.nf;
  Part3 m{0, 0, 0};
#pragma unroll
  for (int p = 0; p < (GRAD ? 16 : 1); ++p) G[p] = 0;
  double Rg = -1e300;
  for (int sl = a.ev_item_off[e] + lane; sl < a.ev_item_off[e + 1]; sl += 64) {
    const double* r = P + (size_t)sl * a.nf;
    const Part3 x{r[0], r[1], r[2]};
    if constexpr (GRAD) {
      if (x.S1 > 0) {
        if (x.R > Rg) {
          for (int p = 0; p < 16; ++p) G[p] = (Rg > -1e299) ? ldexp(G[p], (int)(Rg - x.R)) : 0.0;
          Rg = x.R;
        }
        for (int p = 0; p < 16; ++p) G[p] += ldexp(r[4 + p], (int)(x.R - Rg));
      }
    }
    m = pmerge(m, x);
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const Part3 o{__shfl_xor(m.R, off), __shfl_xor(m.S1, off), __shfl_xor(m.S2, off)};
    m = pmerge(m, o);
    if constexpr (GRAD) {
      const double Ro = __shfl_xor(Rg, off);
      const double Rm = fmax(Rg, Ro);
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        const double go = __shfl_xor(G[p], off);
        G[p] = ((Rg > -1e299) ? ldexp(G[p], (int)(Rg - Rm)) : 0.0) + ((Ro > -1e299) ? ldexp(go, (int)(Ro - Rm)) : 0.0);
      }
      Rg = Rm;
    }
  }
  return m;
}

// Xor butterfly over a wavefront of the combine's partial results: the sums
// of ln L_i, of events used and of their gradient terms G, the flags, and the
// selection's exponent-tracked (R, S1, S2) with its basis sums Gs scaled by
// 2^R.  The sums are commutative and the rescalings exact powers of two, so
// every lane ends with the same bits.
template <bool GRAD>
__device__ __forceinline__ void wave_reduce(double& acc, double& nused, int& fl, double* G, Part3& sel, double* Gs) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    acc += __shfl_xor(acc, off);
    nused += __shfl_xor(nused, off);
    fl |= __shfl_xor(fl, off);
    const Part3 o{__shfl_xor(sel.R, off), __shfl_xor(sel.S1, off), __shfl_xor(sel.S2, off)};
    if constexpr (GRAD) {
      const bool hs = sel.S1 > 0, ho = o.S1 > 0;
      const double Rm = hs && ho ? fmax(sel.R, o.R) : (hs ? sel.R : o.R);
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        G[p] += __shfl_xor(G[p], off);
        const double go = __shfl_xor(Gs[p], off);
        Gs[p] = (hs ? ldexp(Gs[p], (int)(sel.R - Rm)) : 0.0) + (ho ? ldexp(go, (int)(o.R - Rm)) : 0.0);
      }
    }
    sel = pmerge(sel, o);
  }
}

template <bool GRAD>
__device__ void merge_slices(const CombineArgs& a, int b, int n_slices, int lane);

// PRE: each event's items are merged by one wavefront (wave_merge_event);
// otherwise one thread walks an event's items.
template <bool GRAD, bool KDE = false, bool PRE = false>
__global__ __launch_bounds__(256) void combine_kernel(CombineArgs a) {
  static_assert(!(GRAD && KDE), "the KDE numerator has no adjoint");
  static_assert(!(KDE && PRE), "the KDE numerator has its own event records");
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const double ln2 = LN2;
  const double* P = a.part;
  auto at = [&](int slot, int f) { return P[((size_t)b * a.n_items + slot) * a.nf + f]; };
  const bool valid = a.valid[b] != 0;
  double acc = 0;
  double n_ev_used = 0;
  double accg[GRAD ? 16 : 1];
#pragma unroll
  for (int p = 0; p < (GRAD ? 16 : 1); ++p) accg[p] = 0;
  unsigned int flags = 0;
  const int slice = blockIdx.y, n_slices = gridDim.y;
  // an event's ln L_i, N_eff,i and gradient terms from its merged sums m (and
  // the KDE numerator's num); G shares the scale 2^m.R
  auto finish_event = [&](int e, const Part3& m, Part3 num, const double* G) {
    double lnLe, neff;
    if constexpr (!KDE) num = m;
    if (valid && num.S1 > 0) {
      lnLe = log(num.S1) + num.R * ln2 - a.ln_ns[e];
      neff = m.S1 * m.S1 / m.S2;
      if (a.gate_mode == 1 && !(neff >= a.neff_min)) {
        lnLe = -INFINITY;
        flags |= 2u;
      }
    } else {
      lnLe = -INFINITY;
      neff = (valid && m.S1 > 0) ? m.S1 * m.S1 / m.S2 : 0.0;
      flags |= valid ? 2u : 0u;
    }
    if (a.logL_event) a.logL_event[(size_t)b * a.n_events + e] = lnLe;
    if (a.neff_event) a.neff_event[(size_t)b * a.n_events + e] = neff;
    acc += lnLe;
    if constexpr (GRAD) {
      if (m.S1 > 0) {
        for (int p = 0; p < 16; ++p) accg[p] += G[p] / m.S1;
        n_ev_used += 1.0;
      }
    }
  };
  if constexpr (PRE) {
    // wavefront w of slice s takes events s * nw + w, then every n_slices * nw-th
    const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    for (int e = slice * nw + wave; e < a.n_events; e += n_slices * nw) {
      double G[GRAD ? 16 : 1];
      const Part3 m = wave_merge_event<GRAD>(a, b, e, lane, G);
      if (lane == 0) finish_event(e, m, m, G);
    }
  } else {
    for (int e = slice * blockDim.x + tid; e < a.n_events; e += n_slices * blockDim.x) {
      Part3 m{0, 0, 0};
      double G[GRAD ? 16 : 1];
#pragma unroll
      for (int p = 0; p < (GRAD ? 16 : 1); ++p) G[p] = 0;
      double Rg = -1e300;
      Part3 num{0, 0, 0};   // KDE: merged (R, sum of T) of the passing pixels
      if constexpr (KDE) {
        const double* r = a.kde + ((size_t)b * a.n_events + e) * NF_KDE;
        num = Part3{r[0], r[1], 0.0};
        m = Part3{r[0], r[2], r[3]};
      }
      const int sl0 = KDE ? 0 : a.ev_item_off[e];
      const int sl1 = KDE ? 0 : a.ev_item_off[e + 1];
#pragma unroll 4
      for (int sl = sl0; sl < sl1; ++sl) {
        Part3 x{at(sl, 0), at(sl, 1), at(sl, 2)};
        if constexpr (GRAD) {
          if (x.S1 > 0) {
            if (x.R > Rg) {
              for (int p = 0; p < 16; ++p) G[p] = (Rg > -1e299) ? ldexp(G[p], (int)(Rg - x.R)) : 0.0;
              Rg = x.R;
            }
            for (int p = 0; p < 16; ++p) G[p] += ldexp(at(sl, 4 + p), (int)(x.R - Rg));
          }
        }
        m = pmerge(m, x);
      }
      finish_event(e, m, num, G);
    }
  }
  // selection term: strided partial merges, then a fixed tree
  Part3 sel{0, 0, 0};
  double Gs[GRAD ? 16 : 1];
  double Rgs = -1e300;
#pragma unroll
  for (int p = 0; p < (GRAD ? 16 : 1); ++p) Gs[p] = 0;
#pragma unroll 4
  for (int sl = a.inj_slot0 + slice * blockDim.x + tid; sl < a.inj_slot1; sl += n_slices * blockDim.x) {
    Part3 x{at(sl, 0), at(sl, 1), at(sl, 2)};
    if constexpr (GRAD) {
      if (x.S1 > 0) {
        if (x.R > Rgs) {
          for (int p = 0; p < 16; ++p) Gs[p] = (Rgs > -1e299) ? ldexp(Gs[p], (int)(Rgs - x.R)) : 0.0;
          Rgs = x.R;
        }
        for (int p = 0; p < 16; ++p) Gs[p] += ldexp(at(sl, 4 + p), (int)(x.R - Rgs));
      }
    }
    sel = pmerge(sel, x);
  }
  // the block's partial results (256 threads): wavefronts 1-3 leave theirs in
  // LDS, the lanes of wavefront 0 add the three counterparts in order, then an
  // xor butterfly within wavefront 0
  __shared__ double s_acc[256], s_n[256], s_g[GRAD ? 16 : 1][256], s_gs[GRAD ? 16 : 1][256];
  __shared__ int s_fl[256];
  __shared__ Part3 s_sel[256];
  if (tid >= 64) {
    s_acc[tid] = acc;
    s_n[tid] = n_ev_used;
    s_fl[tid] = (int)flags;
    s_sel[tid] = sel;
    if constexpr (GRAD) {
      for (int p = 0; p < 16; ++p) {
        s_g[p][tid] = accg[p];
        s_gs[p][tid] = Gs[p];
      }
    }
  }
  __syncthreads();
  if (tid < 64) {
    int fli = (int)flags;
    for (int t = tid + 64; t < 256; t += 64) {
      acc += s_acc[t];
      n_ev_used += s_n[t];
      fli |= s_fl[t];
      const Part3 o = s_sel[t];
      if constexpr (GRAD) {
        const bool hs = sel.S1 > 0, ho = o.S1 > 0;
        const double Rm = hs && ho ? fmax(sel.R, o.R) : (hs ? sel.R : o.R);
        for (int p = 0; p < 16; ++p) {
          accg[p] += s_g[p][t];
          Gs[p] = (hs ? ldexp(Gs[p], (int)(sel.R - Rm)) : 0.0) + (ho ? ldexp(s_gs[p][t], (int)(o.R - Rm)) : 0.0);
        }
      }
      sel = pmerge(sel, o);
    }
    wave_reduce<GRAD>(acc, n_ev_used, fli, accg, sel, Gs);
    if (tid == 0) {
      if (n_slices == 1) {
        combine_finish<GRAD>(a, b, acc, n_ev_used, (unsigned int)fli, accg, 1, sel, Gs, 1);
      } else {
        // slice record: acc, n_used, flags, selection (R, S1, S2), then 16 + 16 basis sums
        double* o = a.cpart + ((size_t)b * n_slices + slice) * NF_CSLICE;
        o[0] = acc;
        o[1] = n_ev_used;
        o[2] = (double)fli;
        o[3] = sel.R;
        o[4] = sel.S1;
        o[5] = sel.S2;
        if constexpr (GRAD) {
          for (int p = 0; p < 16; ++p) {
            o[6 + p] = accg[p];
            o[22 + p] = Gs[p];
          }
        }
      }
    }
  }
  if (n_slices > 1 && a.slice_ctr) {
    // the point's last slice to finish merges the slice records, in slice
    // order (so the result does not depend on which slice that is); the
    // fences order each slice's record before its count, and the count before
    // the last slice's reads
    __shared__ int last;
    if (tid == 0) {
      __threadfence();
      last = atomicAdd(a.slice_ctr + b, 1) == n_slices - 1;
    }
    __syncthreads();
    if (last && tid < 64) {
      __threadfence();
      merge_slices<GRAD>(a, b, n_slices, tid);
    }
  }
}

// Merge of the slices of one point by one wavefront: lane k takes slices k,
// k + 64, ..., then a fixed xor butterfly.  Its sums are commutative and its
// selection merges exact power-of-two rescalings, so every lane ends with the
// same bits and the result does not depend on timing.
template <bool GRAD>
__device__ void merge_slices(const CombineArgs& a, int b, int n_slices, int lane) {
  double acc = 0, nused = 0;
  int fl = 0;
  Part3 sel{0, 0, 0};
  double G[GRAD ? 16 : 1], Gs[GRAD ? 16 : 1];
#pragma unroll
  for (int p = 0; p < (GRAD ? 16 : 1); ++p) G[p] = Gs[p] = 0;
  for (int sl = lane; sl < n_slices; sl += 64) {
    const double* o = a.cpart + ((size_t)b * n_slices + sl) * NF_CSLICE;
    acc += o[0];
    nused += o[1];
    fl |= (int)o[2];
    const Part3 x{o[3], o[4], o[5]};
    if constexpr (GRAD) {
      for (int p = 0; p < 16; ++p) G[p] += o[6 + p];
      const bool hs = sel.S1 > 0, hx = x.S1 > 0;
      if (hx) {
        const double Rm = hs ? fmax(sel.R, x.R) : x.R;
        for (int p = 0; p < 16; ++p)
          Gs[p] = (hs ? ldexp(Gs[p], (int)(sel.R - Rm)) : 0.0) + ldexp(o[22 + p], (int)(x.R - Rm));
      }
    }
    sel = pmerge(sel, x);
  }
  wave_reduce<GRAD>(acc, nused, fl, G, sel, Gs);
  if (lane == 0) combine_finish<GRAD>(a, b, acc, nused, (unsigned int)fl, G, 1, sel, Gs, 1);
}

// The same merge as a launch of its own (one wavefront per point), for grids
// without slice counters.
template <bool GRAD>
__global__ __launch_bounds__(64) void combine_slices_kernel(CombineArgs a, int n_slices) {
  merge_slices<GRAD>(a, blockIdx.x, n_slices, threadIdx.x);
}

// ---------------------------------------------------------------------------
// sample packing (once per catalogue)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void pack_kernel(const double* __restrict__ m1d, const double* __restrict__ m2d,
                            const double* __restrict__ dl, const double* __restrict__ lnp, int64_t n,
                            Samp<T>* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Samp<T> s;
  const double a = m1d[i], bq = m2d[i];
  s.m1d = (T)a;
  s.m2d = (T)bq;
  s.lm1d = (T)log2(a);
  s.lm2d = (T)log2(bq);
  s.dlc = (T)(dl[i] / C_KMS);
  s.nlp = (T)(-lnp[i] * LOG2E);
  s.lq = (T)log2(bq / a);
  s.dlc_lo = (T)(dl[i] / C_KMS - (double)s.dlc);
  out[i] = s;
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
size_t sweep_lds_bytes(int precision_fp32, int GL, bool grad) {
  const size_t t1 = precision_fp32 ? sizeof(float) : sizeof(double);
  const int NU = precision_fp32 ? NU_F32 : NU_F64, NW = precision_fp32 ? NW_F32 : NW_F64;
  const int NWG = precision_fp32 ? NWG_F32 : NWG_F64;
  return t1 * GL * (2 * (NU + 1) + 2 * (NW + 1) + (grad ? 6 * (NWG + 1) : 0));
}

hipError_t launch_pack(int fp32, const double* m1, const double* m2, const double* dl, const double* lnp,
                       int64_t n, void* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int bs = 256;
  const unsigned gs = (unsigned)((n + bs - 1) / bs);
  if (fp32) pack_kernel<float><<<gs, bs, 0, st>>>(m1, m2, dl, lnp, n, (Samp<float>*)out);
  else pack_kernel<double><<<gs, bs, 0, st>>>(m1, m2, dl, lnp, n, (Samp<double>*)out);
  return hipGetLastError();
}

// threads: per workgroup, 256 ... SETUP_THREADS (the loops stride by the block size).
hipError_t launch_setup(int fp32, const double* lam, int B, double z_max, void* lamc, void* cos_tab,
                        void* win_tab, void* win_grad_tab, int* valid, double* gmap, double* unode, int n_z,
                        int32_t* item_ctr, int threads, hipStream_t st) {
  if (threads < 256 || threads > SETUP_THREADS || threads % 64) return hipErrorInvalidValue;
  if (fp32)
    setup_kernel<float><<<dim3(B, 2), threads, 0, st>>>(lam, B, z_max, (LamC<float>*)lamc, (float2*)cos_tab,
                                      (float2*)win_tab, (float2*)win_grad_tab, valid, gmap, unode, n_z, item_ctr);
  else
    setup_kernel<double><<<dim3(B, 2), threads, 0, st>>>(lam, B, z_max, (LamC<double>*)lamc, (double2*)cos_tab,
                                       (double2*)win_tab, (double2*)win_grad_tab, valid, gmap, unode, n_z, item_ctr);
  return hipGetLastError();
}

template <typename T, int GL, bool GRAD>
static hipError_t sweep_t(const SweepArgs& a, int grid_x, int n_tiles, int threads, size_t lds, hipStream_t st) {
  if (a.z_prior) sweep_kernel<T, GL, GRAD, true><<<dim3(grid_x, n_tiles), threads, lds, st>>>(a);
  else sweep_kernel<T, GL, GRAD, false><<<dim3(grid_x, n_tiles), threads, lds, st>>>(a);
  return hipGetLastError();
}

template <typename T, int GL, bool GRAD>
static hipError_t set_attr(int fp32) {
  const int lds = (int)sweep_lds_bytes(fp32, GL, GRAD);
  hipError_t e = hipFuncSetAttribute((const void*)sweep_kernel<T, GL, GRAD, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)sweep_kernel<T, GL, GRAD, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds);
  return e;
}

// Raise the dynamic-LDS limit of every sweep variant (once, outside any capture).
hipError_t init_kernel_attrs() {
  hipError_t e = hipSuccess;
#define DSL_ATTR(T, G, F)                         \
  if (e == hipSuccess) e = set_attr<T, G, true>(F); \
  if (e == hipSuccess) e = set_attr<T, G, false>(F);
  DSL_ATTR(float, 1, 1)
  DSL_ATTR(float, 4, 1)
  DSL_ATTR(float, 16, 1)
  DSL_ATTR(float, 64, 1)
  DSL_ATTR(double, 1, 0)
  DSL_ATTR(double, 4, 0)
#undef DSL_ATTR
  return e;
}

hipError_t launch_sweep(int fp32, int GL, bool grad, const SweepArgs& a, int grid_x, int threads, hipStream_t st) {
  const int n_tiles = (a.B + GL - 1) / GL;
  const size_t lds = sweep_lds_bytes(fp32, GL, grad);
#define DSL_CASE(T, G)                                                         \
  if (GL == G) return grad ? sweep_t<T, G, true>(a, grid_x, n_tiles, threads, lds, st) \
                           : sweep_t<T, G, false>(a, grid_x, n_tiles, threads, lds, st);
  if (fp32) {
    DSL_CASE(float, 1)
    DSL_CASE(float, 4)
    DSL_CASE(float, 16)
    DSL_CASE(float, 64)
  } else {
    DSL_CASE(double, 1)
    DSL_CASE(double, 4)
  }
#undef DSL_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_gate_split(const GateSplitArgs& a, hipStream_t st) {
  if (a.n_split == 0) return hipSuccess;
  const int64_t n = (int64_t)a.n_split * a.B * 64;   // one wavefront per (split pixel, point)
  gate_split_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_combine(bool grad, const CombineArgs& a, hipStream_t st) {
  const dim3 grid(a.B, a.n_slices);
  if (a.kde) {
    combine_kernel<false, true><<<grid, 256, 0, st>>>(a);
  } else if (a.wave_events) {
    if (grad) combine_kernel<true, false, true><<<grid, 256, 0, st>>>(a);
    else combine_kernel<false, false, true><<<grid, 256, 0, st>>>(a);
  } else if (grad) {
    combine_kernel<true><<<grid, 256, 0, st>>>(a);
  } else {
    combine_kernel<false><<<grid, 256, 0, st>>>(a);
  }
  if (a.n_slices > 1 && !a.slice_ctr) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (grad && !a.kde) combine_slices_kernel<true><<<a.B, 64, 0, st>>>(a, a.n_slices);
    else combine_slices_kernel<false><<<a.B, 64, 0, st>>>(a, a.n_slices);
  }
  return hipGetLastError();
}

}  // namespace dsl
