// HIP kernels (gfx950) of the KDE numerator: the paper's per-pixel weighted
// Gaussian KDE in redshift (Eq. 6) integrated against the pixel's redshift
// prior and the rate on a uniform grid, with the bandwidth rules of Appendix D.
//
//   kde_kernel        one wavefront per (pixel, point): Eq. (7) weights, the
//                     Eq. (8) gate, the bandwidth, the grid integral.
//   kde_event_kernel  one wavefront per (event, point): merge of the event's
//                     passing pixels (read by the combine kernel).
#include "dsl_device.h"

namespace dsl {

// ---------------------------------------------------------------------------
// KDE numerator (Eq. 6 inside Eq. 5; bandwidth rules of Appendix D)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float rdlane(float x, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
}
__device__ __forceinline__ int rdlane(int x, int j) { return __builtin_amdgcn_readlane(x, j); }
__device__ __forceinline__ double rdlane(double x, int j) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), j);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Cross-lane moves inside the DPP row patterns of gfx9: lane i of the result
// takes x from the lane the control selects; rows outside ROWS receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp32(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp32<CTRL, ROWS>((int)(b & 0xffffffff));
  const int hi = dpp32<CTRL, ROWS>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(dpp32<CTRL, ROWS>(__float_as_int(x)));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp(int x) {
  return dpp32<CTRL, ROWS>(x);
}

// Reduction over the 64 lanes of a wavefront (every lane active), returned to
// all lanes: pairs and quads (quad_perm), half rows (row_half_mirror), rows
// (row_mirror), then rows 0+1 and 2+3 (row_bcast:15) and all four rows
// (row_bcast:31), read from lane 63.  The order is fixed, so it is deterministic.
template <typename V, typename Op>
__device__ __forceinline__ V wave_reduce(V x, Op op) {
  x = op(x, dpp<0xB1, 0xf>(x));    // quad_perm [1,0,3,2]
  x = op(x, dpp<0x4E, 0xf>(x));    // quad_perm [2,3,0,1]
  x = op(x, dpp<0x141, 0xf>(x));   // row_half_mirror
  x = op(x, dpp<0x140, 0xf>(x));   // row_mirror
  x = op(x, dpp<0x142, 0xa>(x));   // row_bcast:15 into rows 1 and 3
  x = op(x, dpp<0x143, 0xc>(x));   // row_bcast:31 into rows 2 and 3
  return rdlane(x, 63);
}
__device__ __forceinline__ double wave_sum(double x) {
  return wave_reduce(x, [](double a, double b) { return a + b; });
}

// Reduction over each 16-lane row (pairs, quads, half rows, rows): every lane
// of a row ends with its row's result; rows do not mix.
template <typename V, typename Op>
__device__ __forceinline__ V row_reduce(V x, Op op) {
  x = op(x, dpp<0xB1, 0xf>(x));    // quad_perm [1,0,3,2]
  x = op(x, dpp<0x4E, 0xf>(x));    // quad_perm [2,3,0,1]
  x = op(x, dpp<0x141, 0xf>(x));   // row_half_mirror
  x = op(x, dpp<0x140, 0xf>(x));   // row_mirror
  return x;
}

// Linear interpolation of a redshift-prior row at z in [0, z_max].
template <typename T>
__device__ __forceinline__ T los_at(const T* __restrict__ row, int n_z, T inv_dz, T z) {
  const T x = z * inv_dz;
  int k = (int)x;
  k = k < 0 ? 0 : (k > n_z - 2 ? n_z - 2 : k);
  const T f = x - (T)k;
  const T l0 = (T)row[k], l1 = (T)row[k + 1];
  return l0 + f * (l1 - l0);
}

// psi(z)/(1+z) = (1+z)^(gamma-1) / (1 + ((1+z)/(1+z_p))^(gamma+kappa)) without its constant.
template <typename T>
__device__ __forceinline__ T rate_at(const LamC<T>& c, T z) {
  using M = Mth<T>;
  const T L = M::log2((T)1 + z);
  const T eX = c.gk * (L - c.Lp);
  return M::exp2((c.gm3 + (T)2) * L - fmax(eX, (T)0)) * M::rcp((T)1 + M::exp2(-fabs(eX)));
}

// Row kernel (fewer than four points per call, the paper's one point per
// evaluation): each 16-lane DPP row of a wavefront serves one (pixel part,
// point) pair -- four consecutive pairs per wavefront, pixel-major, so no row
// idles -- and reduces its own sums (no cross-row traffic).  Pass A (the row's
// lanes stride over the samples): Eq. (7) weights without prior and rate,
// Eq. (8) sums, in-support redshift moments and range.  Bandwidth from the
// in-support redshifts (order statistics in ascending d_L order, which is
// ascending z for any point).  Pass B (each lane holds 16 consecutive grid
// nodes of its point per block of 256 nodes): f(z_g) = sum_k w_k
// exp(-(z_g - z_k)^2 / 2h^2) over the row's samples (by the node-to-node ratio
// recurrence of a Gaussian on a uniform grid), then T = dz / (h sqrt(2 pi)) *
// sum_g c_g p_LOS(z_g) rate(z_g) f(z_g) with trapezoid weights c_g.
// FP32: 4 waves per SIMD (a few registers spill; measured faster than 3 waves
// without spills); FP64: 2.
template <typename T> struct KdeWaves { static constexpr int W = 4; };
template <> struct KdeWaves<double> { static constexpr int W = 2; };

// SPLIT: tasks are pixel parts (a.parts) whose grid stage covers samples
// [lo, hi) of the pixel; otherwise one part per pixel.
template <typename T, int LT, bool SPLIT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(KdeWaves<T>::W))) void kde_kernel(KdeArgs a) {
  using T2 = typename V2<T>::t;
  constexpr int NU = Tab<T>::NU, NW = Tab<T>::NW;
  constexpr int NB = 16;   // grid nodes per lane per block of 256 nodes
  extern __shared__ __align__(16) unsigned char smem[];
  // block work counters: (sample, node) kernel terms, grid nodes evaluated
  __shared__ unsigned long long work[2];
  if (threadIdx.x < 2) work[threadIdx.x] = 0ull;
  T2* cosL = reinterpret_cast<T2*>(smem);
  T2* winL = cosL + (NU + 1) * LT;
  const int tile = blockIdx.y;
  const int nl = a.B - tile * LT < LT ? a.B - tile * LT : LT;
  const T2* cos_g = reinterpret_cast<const T2*>(a.cos_tab);
  const T2* win_g = reinterpret_cast<const T2*>(a.win_tab);
  for (int i = threadIdx.x; i < (NU + 1) * LT; i += blockDim.x) {
    const int k = i / LT, l = i % LT, b = tile * LT + l;
    cosL[i] = l < nl ? cos_g[(size_t)b * (NU + 1) + k] : T2{};
  }
  for (int i = threadIdx.x; i < (NW + 1) * LT; i += blockDim.x) {
    const int k = i / LT, l = i % LT, b = tile * LT + l;
    winL[i] = l < nl ? win_g[(size_t)b * (NW + 1) + k] : T2{};
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4, kl = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;
  const LamC<T>* lamc = reinterpret_cast<const LamC<T>*>(a.lamc);
  const Samp<T>* __restrict__ samp = reinterpret_cast<const Samp<T>*>(a.samp);
  const TabView<T> tv{cosL, winL, nullptr};
  const T inv_dz = (T)((a.n_z - 1) / a.z_max);
  const int64_t n_units = SPLIT ? a.n_parts : a.n_pix;   // pixel parts, or whole pixels
  const int64_t n_pairs = n_units * nl;
  const int64_t n_tasks = (n_pairs + 3) / 4;
  for (int64_t t = (int64_t)blockIdx.x * nwaves + wave; t < n_tasks; t += (int64_t)gridDim.x * nwaves) {
    // this row's pixel part and point in the tile
    const int64_t i = 4 * t + q;
    const bool act = i < n_pairs;
    const int64_t pi = act ? i / nl : 0;
    const int l = act ? (int)(i - pi * nl) : 0;
    KdePart part{pi, 0, 0};
    if constexpr (SPLIT) part = a.parts[pi];
    const int64_t p = part.pix;
    const int b = tile * LT + (act ? l : 0);
    const LamC<T> c = lamc[b];
    const bool live = act && c.valid;
    double* out = a.out + ((size_t)b * n_units + pi) * NF_KDE;
    const int64_t s0 = a.pix_off[p];
    // pass A and the bandwidth take the whole pixel, the grid stage [lo, hi)
    const int n = act ? (int)(a.pix_off[p + 1] - s0) : 0;
    const int lo = SPLIT && act ? part.lo : 0;
    const int hi = SPLIT && act ? (part.hi < n ? part.hi : n) : n;
    // ---- pass A
    PixAcc<false, T> pa;
    pa.zero();
    double sz = 0.0, szz = 0.0;   // in-support redshift moments
    T zlo = (T)INFINITY, zhi = (T)-INFINITY;
    int cin = 0;
    T z1 = (T)-1, lin1 = (T)0;    // the lane's sample when n <= 16
    int ne1 = R_SENTINEL;
    for (int c0 = 0; c0 < n; c0 += 16) {
      const int k = c0 + kl;
      if (k < n && live) {
        int ne;
        T lin, z;
        eval_weight<T, LT, false, true>(samp[s0 + k], c, tv, l, nullptr, 0, (T)0, ne, lin, nullptr, &z);
        pa.template add<T>(ne, lin, nullptr);
        if (z >= (T)0) {
          sz += (double)z;
          szz += (double)z * (double)z;
          zlo = fmin(zlo, z);
          zhi = fmax(zhi, z);
          ++cin;
        }
        z1 = z;
        lin1 = lin;
        ne1 = ne;
      }
    }
    const int R = row_reduce(pa.R, [](int x, int y) { return x > y ? x : y; });
    const double S1 = row_reduce(ldexp(pa.S1, pa.R - R), [](double x, double y) { return x + y; });
    const double S2 = row_reduce(ldexp(pa.S2, 2 * (pa.R - R)), [](double x, double y) { return x + y; });
    bool pass;
    if (a.gate_mode == 2) pass = live && S1 > 0;
    else pass = live && S2 > 0 && S1 * S1 >= a.neff_min * S2;
    // the in-support moments and range serve only the bandwidth of a passing
    // row (pass is uniform over a row, and every reduction stays in its row)
    int nin = 0;
    if (pass) {
      sz = row_reduce(sz, [](double x, double y) { return x + y; });
      szz = row_reduce(szz, [](double x, double y) { return x + y; });
      zlo = row_reduce(zlo, [](T x, T y) { return fmin(x, y); });
      zhi = row_reduce(zhi, [](T x, T y) { return fmax(x, y); });
      nin = row_reduce(cin, [](int x, int y) { return x + y; });
    }
    // ---- bandwidth (Appendix D) from the n_in in-support redshifts of the row's point
    auto zs = [&](int r) -> double {   // r-th smallest in-support redshift
      const Samp<T> sp = samp[s0 + a.perm[s0 + r]];
      return (double)z_of_u<T, LT>(fma(sp.dlc, c.H0, sp.dlc * c.H0_lo), c, tv, l);
    };
    // the lane's redshift and scaled weight in the chunk from c0 (samples below lim)
    auto z_w = [&](int c0, int lim, T& z, T& w) {
      if (n <= 16) {
        z = z1;
        w = (z1 >= (T)0 && lin1 > (T)0) ? ldexp(lin1, ne1 - R) : (T)0;
        return;
      }
      const int k = c0 + kl;
      z = (T)-1;
      w = (T)0;
      if (k < lim && live) {
        int ne;
        T lin;
        eval_weight<T, LT, false, true>(samp[s0 + k], c, tv, l, nullptr, 0, (T)0, ne, lin, nullptr, &z);
        if (z >= (T)0 && lin > (T)0) w = ldexp(lin, ne - R);
      }
    };
    double h = 0.0;
    if (pass && nin >= 2 && zlo < zhi) {   // equal redshifts: zero spread, zero bandwidth
      const double sd = sqrt(fmax(szz - sz * sz / (double)nin, 0.0) / (double)(nin - 1));
      const double nf = (double)Mth<T>::exp2((T)-0.2 * Mth<T>::log2((T)nin));   // n^(-1/5)
      if (a.bandwidth == 0) {
        h = 1.06 * sd * nf;
      } else if (a.bandwidth == 1) {
        auto qt = [&](double pr) {
          const double pos = pr * (double)(nin - 1);
          const int i0 = (int)floor(pos);
          const int i1 = i0 + 1 < nin ? i0 + 1 : nin - 1;
          const double z0 = zs(i0);
          return z0 + (pos - (double)i0) * (zs(i1) - z0);
        };
        h = 0.9 * fmin(sd, (qt(0.75) - qt(0.25)) / 1.34) * nf;
      } else {
        const int m = (nin - 1) / 2;
        const double Q = 0.5 * (zs(m) + zs(nin / 2));
        const int nA = m + 1, nB = nin - m - 1;
        // k-th smallest deviation: A_i = Q - z_(m-i) and B_i = z_(m+1+i) - Q are
        // both ascending; binary search on how many come from A.
        auto kth = [&](int k) -> double {
          int lo = k + 1 - nB > 0 ? k + 1 - nB : 0;
          int hi = k + 1 < nA ? k + 1 : nA;
          while (lo < hi) {
            const int i = (lo + hi) >> 1, j = k + 1 - i;
            if (Q - zs(m - i) < zs(m + j) - Q) lo = i + 1;
            else hi = i;
          }
          const int j = k + 1 - lo;
          double v = -INFINITY;
          if (lo > 0) v = fmax(v, Q - zs(m - lo + 1));
          if (j > 0) v = fmax(v, zs(m + j) - Q);
          return v;
        };
        const double mad = 0.5 * (kth((nin - 1) / 2) + kth(nin / 2));
        if (mad > 0.0) {
          const double iu = 1.0 / (9.0 * mad);
          double num = 0.0, den = 0.0;
          for (int c0 = 0; c0 < n; c0 += 16) {
            T z, w;
            z_w(c0, n, z, w);
            if (z >= (T)0) {
              const double d = (double)z - Q, u = d * iu, uu = u * u;
              if (fabs(u) < 1.0) {
                const double om = 1.0 - uu;
                num += d * d * (om * om) * (om * om);
                den += om * (1.0 - 5.0 * uu);
              }
            }
          }
          num = row_reduce(num, [](double x, double y) { return x + y; });
          den = row_reduce(den, [](double x, double y) { return x + y; });
          const double bm = (double)nin * num / (den * den);
          h = bm > 0.0 ? 1.06 * sqrt(bm) * nf : 0.0;
        }
      }
    }
    const T* __restrict__ row = reinterpret_cast<const T*>(a.los) + (size_t)a.pix_row[p] * a.n_z;
    const bool kde_row = pass && h > 0.0 && isfinite(h);
    double Tt = 0.0;
    if (pass && !kde_row) {
      // zero bandwidth: point masses at the part's samples
      for (int c0 = lo; c0 < hi; c0 += 16) {
        T z, w;
        z_w(c0, hi, z, w);
        if (w > (T)0) Tt += (double)w * (double)(los_at<T>(row, a.n_z, inv_dz, z) * rate_at<T>(c, z));
      }
      Tt = row_reduce(Tt, [](double x, double y) { return x + y; });
    } else if (kde_row) {
      // ---- pass B
      const double ga = fmax(0.0, (double)zlo - a.tau * h);
      const double gb = fmin(a.z_max, (double)zhi + a.tau * h);
      const double dz = (gb - ga) / (double)(a.n_grid - 1);
      // coordinates scaled by sqrt(log2(e)/2)/h and measured from ga, so each
      // term is exp2(-(x_g - x_k)^2); S is the node spacing in these units
      const T invh = (T)(sqrt(0.5 * LOG2E) / h);
      const T S = (T)(dz * (sqrt(0.5 * LOG2E) / h));
      // Each lane holds NB consecutive nodes.  With x_g = x_0 + i S the terms
      // of one sample follow t_i = u_i C_i, u_i = u_{i-1} P, C_i = 2^(-(i S)^2),
      // P = 2^(-2 S (x_0 - x_k)), u_0 = w_k t_0: C_i goes into the node factor,
      // so a term costs a multiply and an add.  u_i <= w_k 2^((NB-1)^2 S^2), and
      // P is formed as 2^(-2 S x_0) 2^(2 S x_k) with both factors within
      // 2^(+-2 S^2 (n_grid - 1)), so the recurrence is used while S <= 1/4 and
      // 2 S^2 (n_grid - 1) <= 64 (row-uniform); wider spacings (a grid coarser
      // than about a third of the bandwidth) evaluate every term.
      const bool rec = S <= (T)0.25 && (T)2 * S * S * (T)(a.n_grid - 1) <= (T)64;
      // psi(z)/(1+z) = 1 / (2^(-(gamma-1) L) + 2^((kappa+1) L - (gamma+kappa) L_p)), L = log2(1+z)
      const T ra = -(c.gm3 + (T)2), rb = c.gk - (c.gm3 + (T)2), rc = -c.gk * c.Lp;
      const unsigned nz2 = (unsigned)(a.n_z - 2);
      if (kl == 0 && a.evals && lo == 0) atomicAdd(&work[1], (unsigned long long)a.n_grid);
      for (int g0 = 0; g0 < a.n_grid; g0 += 16 * NB) {
        T vg[NB];
        // Node g = g0 + NB kl + i.  Trapezoid weight min(max(n_grid - 1/2 - g, 0), 1):
        // 1 inside, 1/2 at the last node, 0 past the end (the first node is halved below).
        const int gl = g0 + NB * kl;
        double zd = ga + (double)gl * dz;
        const T cw = (T)a.n_grid - (T)0.5 - (T)gl;
        const T x0l = (T)((double)gl * dz) * invh;
        // C_i = 2^(-(i S)^2) by C_{i+1} = C_i r_i, r_i = 2^(-(2i+1) S^2), r_{i+1} = r_i 2^(-2 S^2)
        const T r0 = Mth<T>::exp2(-(S * S));
        const T r2 = r0 * r0;
        T Ci = (T)1, ri = r0;
        // the table loads of LB nodes are issued before their arithmetic
        constexpr int LB = 8;
#pragma unroll
        for (int i0 = 0; i0 < NB; i0 += LB) {
          T lp0[LB], lp1[LB];
          T zgv[LB], fz[LB];
#pragma unroll
          for (int i = 0; i < LB; ++i) {
            const T zg = (T)fmin(zd, a.z_max);
            zd += dz;
            const T x = zg * inv_dz;   // zg >= 0
            unsigned k = (unsigned)x;
            k = k < nz2 ? k : nz2;
            zgv[i] = zg;
            fz[i] = x - (T)k;
            los_pair(row, k, lp0[i], lp1[i]);
          }
#pragma unroll
          for (int i = 0; i < LB; ++i) {
            const int ii = i0 + i;
            const T zg = zgv[i];
            const T cg = fmin(fmax(cw - (T)ii, (T)0), (T)1);
            const T L = Mth<T>::log2((T)1 + zg);
            const T rate = Mth<T>::rcp(Mth<T>::exp2(ra * L) + Mth<T>::exp2(fma(rb, L, rc)));
            const T l0 = lp0[i], l1 = lp1[i];
            vg[ii] = cg * rate * (l0 + fz[i] * (l1 - l0)) * (rec ? Ci : (T)1);
            Ci *= ri;
            ri *= r2;
          }
        }
        if (g0 == 0 && kl == 0) vg[0] *= (T)0.5;
        const T A = Mth<T>::exp2((T)-2 * S * x0l);
        for (int c0 = lo; c0 < hi; c0 += 16) {
          T z, w;
          z_w(c0, hi, z, w);
          // out-of-support samples (z = -1) carry w = 0 and give exact zeros
          const T zr = (z - (T)ga) * invh;
          const T Bk = Mth<T>::exp2((T)2 * S * zr);
          const int cnt = hi - c0 < 16 ? hi - c0 : 16;
          if (g0 == 0) {
            const unsigned long long m = __ballot(w > (T)0);
            if (kl == 0 && a.evals)
              atomicAdd(&work[0], (unsigned long long)__popcll((m >> (16 * q)) & 0xffffull) * a.n_grid);
          }
          T accf[NB];
#pragma unroll
          for (int i = 0; i < NB; ++i) accf[i] = (T)0;
          int j = 0;
          if (rec) {
            do {   // cnt >= 1
              const T wj = __shfl(w, j, 16);
              const T zj = __shfl(zr, j, 16);
              const T P = A * __shfl(Bk, j, 16);
              const T x0 = x0l - zj;
              T u = wj * Mth<T>::exp2(-(x0 * x0));
              accf[0] += u;
#pragma unroll
              for (int i = 1; i < NB; ++i) {
                u *= P;
                accf[i] += u;
              }
            } while (++j < cnt);
          } else {
            do {
              const T wj = __shfl(w, j, 16);
              const T zj = __shfl(zr, j, 16);
#pragma unroll
              for (int i = 0; i < NB; ++i) {
                const T xx = fma((T)i, S, x0l) - zj;
                accf[i] = fma(wj, Mth<T>::exp2(-(xx * xx)), accf[i]);
              }
            } while (++j < cnt);
          }
          // the lane's 16 positive terms of this chunk in T, the running sum in FP64
          T part = (T)0;
#pragma unroll
          for (int i = 0; i < NB; ++i) part = fma(vg[i], accf[i], part);
          Tt += (double)part;
        }
      }
      Tt = row_reduce(Tt, [](double x, double y) { return x + y; }) * dz / (h * 2.5066282746310002);
    }
    if (act && kl == 0) {
      out[0] = pass ? (double)R : 0.0;
      out[1] = pass ? Tt : 0.0;
      out[2] = pass && lo == 0 ? S1 : 0.0;
      out[3] = pass && lo == 0 ? S2 : 0.0;
    }
  }
  __syncthreads();
  if (a.evals && threadIdx.x < 2 && work[threadIdx.x]) atomicAdd(a.evals + threadIdx.x, work[threadIdx.x]);
}

// k-th set bit (from 0) of a mask holding more than k set bits: the largest
// position whose lower bits hold at most k set bits.
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int k) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w > 0; w >>= 1)
    if (__popcll(m & ((1ull << (pos + w)) - 1ull)) <= k) pos += w;
  return pos;
}

// Batched KDE numerator (four or more points): one wavefront per (pixel, tile
// of GL points), pixels largest first.  Pass A in the sweep's layout: GL points
// x 64/GL sample groups per wavefront (GL = 64: one lane per point, each sample
// record loaded once for the tile from a uniform address); Eq. (7) weights
// without prior and rate, Eq. (8) sums, in-support redshift moments and range,
// the gate and the bandwidth of every point at once.  Grid stage: the points of
// the pixel that pass are packed into the wavefront's four 16-lane rows, four
// per round (only a pixel's last round leaves rows idle); each row computes
// its point's T as the row kernel does, re-evaluating the pixel's samples.
// Records {R, T, S1, S2} per (pixel, point), T = 0 for failing pairs.
template <typename T> struct KdeTileThreads { static constexpr int N = 256 * KdeWaves<T>::W; };

template <typename T, int GL>
__global__ __launch_bounds__(KdeTileThreads<T>::N) __attribute__((amdgpu_waves_per_eu(KdeWaves<T>::W))) void
kde_tile_kernel(KdeArgs a) {
  using T2 = typename V2<T>::t;
  constexpr int NU = Tab<T>::NU, NW = Tab<T>::NW;
  constexpr int NS = 64 / GL;   // sample groups per point
  constexpr int NB = 16;        // grid nodes per lane per block of 256 nodes
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ unsigned long long work[2];
  if (threadIdx.x < 2) work[threadIdx.x] = 0ull;
  T2* cosL = reinterpret_cast<T2*>(smem);
  T2* winL = cosL + (NU + 1) * GL;
  LamC<T>* lamL = reinterpret_cast<LamC<T>*>(winL + (NW + 1) * GL);
  const int tile = blockIdx.y;
  const int nl = a.B - tile * GL < GL ? a.B - tile * GL : GL;
  const T2* cos_g = reinterpret_cast<const T2*>(a.cos_tab);
  const T2* win_g = reinterpret_cast<const T2*>(a.win_tab);
  const LamC<T>* lamc = reinterpret_cast<const LamC<T>*>(a.lamc);
  for (int i = threadIdx.x; i < (NU + 1) * GL; i += blockDim.x) {
    const int k = i / GL, l = i % GL, b = tile * GL + l;
    cosL[i] = l < nl ? cos_g[(size_t)b * (NU + 1) + k] : T2{};
  }
  for (int i = threadIdx.x; i < (NW + 1) * GL; i += blockDim.x) {
    const int k = i / GL, l = i % GL, b = tile * GL + l;
    winL[i] = l < nl ? win_g[(size_t)b * (NW + 1) + k] : T2{};
  }
  for (int i = threadIdx.x; i < GL; i += blockDim.x) lamL[i] = lamc[tile * GL + (i < nl ? i : 0)];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;
  const int lam = lane % GL, sg = lane / GL;
  const int q = lane >> 4, kl = lane & 15;
  const bool act = lam < nl;
  // (the lane's point constants are read from LDS per task: registers stay free for the grid stage)
  const bool live = act && lamL[lam].valid;
  const Samp<T>* __restrict__ samp = reinterpret_cast<const Samp<T>*>(a.samp);
  const T* __restrict__ los = reinterpret_cast<const T*>(a.los);
  const TabView<T> tv{cosL, winL, nullptr};
  const T inv_dz = (T)((a.n_z - 1) / a.z_max);
  // Pixels in batches of KDE_PIX_BATCH, batch b holding the b-th pixel of each
  // of KDE_PIX_BATCH equal strata of the largest-first order (so no batch
  // gathers the largest pixels): each wavefront's first batch by a fixed
  // stride, the rest from the tile's counter (by a stride, the largest-first
  // order would give the same workgroups the largest pixels of every round);
  // every pixel writes its own record, so the results do not depend on which
  // wavefront took it.
  constexpr int PB = KDE_PIX_BATCH;
  const int64_t n_bat = (a.n_pix + PB - 1) / PB;
  const int64_t n_first = (int64_t)gridDim.x * nwaves;
  int32_t* const ctr = a.pix_ctr && n_first < n_bat ? a.pix_ctr + tile : nullptr;
  auto next_batch = [&](int64_t bt) -> int64_t {
    if (!ctr) return bt + n_first;
    int v = 0;
    if (lane == 0) v = atomicAdd(ctr, 1);
    return n_first + __builtin_amdgcn_readfirstlane(v);
  };
  for (int64_t bt = (int64_t)blockIdx.x * nwaves + wave; bt < n_bat; bt = next_batch(bt)) {
    for (int64_t t = bt; t < a.n_pix; t += n_bat) {
      // (pixel and bounds are the same on every lane: scalars keep pass A's
      // loop counter and record addresses off the vector unit)
      const int64_t p = uniform64(a.order ? (int64_t)a.order[t] : t);
      const LamC<T>& c = lamL[lam];
      const int64_t s0 = uniform64(a.pix_off[p]);
      const int n = (int)(uniform64(a.pix_off[p + 1]) - s0);
      // ---- pass A (the next record is loaded while the current one is evaluated)
      PixAcc<false, T> pa;
      pa.zero();
      double sz = 0.0, szz = 0.0;
      T zlo = (T)INFINITY, zhi = (T)-INFINITY;
      int cin = 0;
      if (n > 0) {
        auto at = [&](int k) { const int i = k + sg; return s0 + (i < n ? i : n - 1); };
        Samp<T> nxt = ld_samp<T, NS>(samp, at(0));
        for (int k0 = 0; k0 < n; k0 += NS) {
          const Samp<T> cur = nxt;
          if (k0 + NS < n) nxt = ld_samp<T, NS>(samp, at(k0 + NS));
          if (k0 + sg < n && live) {
            int ne;
            T lin, z;
            eval_weight<T, GL, false, true>(cur, c, tv, lam, nullptr, 0, (T)0, ne, lin, nullptr, &z);
            pa.template add<T>(ne, lin, nullptr);
            if (z >= (T)0) {
              sz += (double)z;
              szz += (double)z * (double)z;
              zlo = fmin(zlo, z);
              zhi = fmax(zhi, z);
              ++cin;
            }
          }
        }
      }
      // sample groups of a point merged by a fixed xor tree (commutative merges:
      // every lane of a point ends with the same bits)
  #pragma unroll
      for (int off = GL; off < 64; off <<= 1) {
        pa.xor_merge(off);
        sz += __shfl_xor(sz, off);
        szz += __shfl_xor(szz, off);
        zlo = fmin(zlo, __shfl_xor(zlo, off));
        zhi = fmax(zhi, __shfl_xor(zhi, off));
        cin += __shfl_xor(cin, off);
      }
      const int R = pa.R;
      bool pass;
      if (a.gate_mode == 2) pass = live && pa.S1 > 0;
      else pass = live && pa.S2 > 0 && pa.S1 * pa.S1 >= a.neff_min * pa.S2;
      // ---- bandwidth (Appendix D) of each point, from its nin in-support redshifts
      const int nin = cin;
      // z of the sample of local index k, -1 beyond the support (point of this lane)
      auto z_of = [&](int64_t k) -> T {
        const Samp<T> sp = samp[s0 + k];
        const T u = fma(sp.dlc, c.H0, sp.dlc * c.H0_lo);
        return u <= c.u_max ? z_of_u<T, GL>(u, c, tv, lam) : (T)-1;
      };
      auto zs = [&](int r) -> double { return (double)z_of(a.perm[s0 + r]); };   // r-th smallest in-support z
      double h = 0.0;
      if (pass && nin >= 2 && zlo < zhi) {
        const double sd = sqrt(fmax(szz - sz * sz / (double)nin, 0.0) / (double)(nin - 1));
        const double nf = (double)Mth<T>::exp2((T)-0.2 * Mth<T>::log2((T)nin));   // n^(-1/5)
        if (a.bandwidth == 0) {
          h = 1.06 * sd * nf;
        } else if (a.bandwidth == 1) {
          auto qt = [&](double pr) {
            const double pos = pr * (double)(nin - 1);
            const int i0 = (int)floor(pos);
            const int i1 = i0 + 1 < nin ? i0 + 1 : nin - 1;
            const double z0 = zs(i0);
            return z0 + (pos - (double)i0) * (zs(i1) - z0);
          };
          h = 0.9 * fmin(sd, (qt(0.75) - qt(0.25)) / 1.34) * nf;
        }
      }
      if (a.bandwidth == 2) {
        // biweight: median and MAD by order statistics, then the midvariance sums
        // over the samples (sample groups merged like pass A)
        const bool bw = pass && nin >= 2 && zlo < zhi;
        double Q = 0.0, mad = 0.0;
        if (bw) {
          const int m = (nin - 1) / 2;
          Q = 0.5 * (zs(m) + zs(nin / 2));
          const int nA = m + 1, nB = nin - m - 1;
          // k-th smallest deviation: A_i = Q - z_(m-i) and B_i = z_(m+1+i) - Q are
          // both ascending; binary search on how many come from A
          auto kth = [&](int k) -> double {
            int lo = k + 1 - nB > 0 ? k + 1 - nB : 0;
            int hi = k + 1 < nA ? k + 1 : nA;
            while (lo < hi) {
              const int i = (lo + hi) >> 1, j = k + 1 - i;
              if (Q - zs(m - i) < zs(m + j) - Q) lo = i + 1;
              else hi = i;
            }
            const int j = k + 1 - lo;
            double v = -INFINITY;
            if (lo > 0) v = fmax(v, Q - zs(m - lo + 1));
            if (j > 0) v = fmax(v, zs(m + j) - Q);
            return v;
          };
          mad = 0.5 * (kth((nin - 1) / 2) + kth(nin / 2));
        }
        double num = 0.0, den = 0.0;
        if (bw && mad > 0.0) {
          const double iu = 1.0 / (9.0 * mad);
          for (int k = sg; k < n; k += NS) {
            const T z = z_of(k);
            if (z >= (T)0) {
              const double d = (double)z - Q, u = d * iu, uu = u * u;
              if (fabs(u) < 1.0) {
                const double om = 1.0 - uu;
                num += d * d * (om * om) * (om * om);
                den += om * (1.0 - 5.0 * uu);
              }
            }
          }
        }
  #pragma unroll
        for (int off = GL; off < 64; off <<= 1) {
          num += __shfl_xor(num, off);
          den += __shfl_xor(den, off);
        }
        if (bw && mad > 0.0) {
          const double nf = (double)Mth<T>::exp2((T)-0.2 * Mth<T>::log2((T)nin));
          const double bm = (double)nin * num / (den * den);
          h = bm > 0.0 ? 1.06 * sqrt(bm) * nf : 0.0;
        }
      }
      const bool kde_row = pass && h > 0.0 && isfinite(h);
      if (sg == 0 && act) {
        // (T of a passing pair is written by its row in the grid stage)
        double* out = a.out + ((size_t)(tile * GL + lam) * a.n_pix + p) * NF_KDE;
        out[0] = pass ? (double)R : 0.0;
        if (!pass) out[1] = 0.0;
        out[2] = pass ? pa.S1 : 0.0;
        out[3] = pass ? pa.S2 : 0.0;
      }
      // ---- grid stage: the passing points, four per round, one 16-lane row each
      const unsigned long long pm = __ballot(sg == 0 && pass);
      const int np = __popcll(pm);
      const T* __restrict__ row = los + (size_t)a.pix_row[p] * a.n_z;
      for (int r0 = 0; r0 < np; r0 += 4) {
        const int kq = r0 + q;
        const bool ract = kq < np;
        const int src = ract ? nth_set_bit(pm, kq) : 0;   // a lane with sg = 0: its point is lam = src
        const int lp = src;
        const int Rp = __shfl(R, src);
        const double hp = __shfl(h, src);
        const T zlop = __shfl(zlo, src), zhip = __shfl(zhi, src);
        const bool krow = __shfl((int)kde_row, src) != 0;
        const LamC<T>& cp = lamL[lp];
        // the lane's redshift and scaled weight of sample c0 + kl (samples below lim)
        auto z_w = [&](int c0, int lim, T& z, T& w) {
          const int k = c0 + kl;
          z = (T)-1;
          w = (T)0;
          if (k < lim && ract) {
            int ne;
            T lin;
            eval_weight<T, GL, false, true>(samp[s0 + k], cp, tv, lp, nullptr, 0, (T)0, ne, lin, nullptr, &z);
            if (z >= (T)0 && lin > (T)0) w = ldexp(lin, ne - Rp);
          }
        };
        double Tt = 0.0;
        if (ract && !krow) {
          // zero bandwidth: point masses at the samples
          for (int c0 = 0; c0 < n; c0 += 16) {
            T z, w;
            z_w(c0, n, z, w);
            if (w > (T)0) Tt += (double)w * (double)(los_at<T>(row, a.n_z, inv_dz, z) * rate_at<T>(cp, z));
          }
          Tt = row_reduce(Tt, [](double x, double y) { return x + y; });
        } else if (ract) {
          const double ga = fmax(0.0, (double)zlop - a.tau * hp);
          const double gb = fmin(a.z_max, (double)zhip + a.tau * hp);
          const double dz = (gb - ga) / (double)(a.n_grid - 1);
          // coordinates scaled by sqrt(log2(e)/2)/h and measured from ga, so each
          // term is exp2(-(x_g - x_k)^2); S is the node spacing in these units;
          // the node-to-node ratio recurrence as in the row kernel
          const T invh = (T)(sqrt(0.5 * LOG2E) / hp);
          const T S = (T)(dz * (sqrt(0.5 * LOG2E) / hp));
          const bool rec = S <= (T)0.25 && (T)2 * S * S * (T)(a.n_grid - 1) <= (T)64;
          const T ra = -(cp.gm3 + (T)2), rb = cp.gk - (cp.gm3 + (T)2), rc = -cp.gk * cp.Lp;
          const unsigned nz2 = (unsigned)(a.n_z - 2);
          if (kl == 0 && a.evals) atomicAdd(&work[1], (unsigned long long)a.n_grid);
          for (int g0 = 0; g0 < a.n_grid; g0 += 16 * NB) {
            T vg[NB];
            const int gl = g0 + NB * kl;
            double zd = ga + (double)gl * dz;
            const T cw = (T)a.n_grid - (T)0.5 - (T)gl;
            const T x0l = (T)((double)gl * dz) * invh;
            const T r0 = Mth<T>::exp2(-(S * S));
            const T r2 = r0 * r0;
            T Ci = (T)1, ri = r0;
            constexpr int LB = 8;
  #pragma unroll
            for (int i0 = 0; i0 < NB; i0 += LB) {
              T lp0[LB], lp1[LB];
              T zgv[LB], fz[LB];
  #pragma unroll
              for (int i = 0; i < LB; ++i) {
                const T zg = (T)fmin(zd, a.z_max);
                zd += dz;
                const T x = zg * inv_dz;
                unsigned k = (unsigned)x;
                k = k < nz2 ? k : nz2;
                zgv[i] = zg;
                fz[i] = x - (T)k;
                los_pair(row, k, lp0[i], lp1[i]);
              }
  #pragma unroll
              for (int i = 0; i < LB; ++i) {
                const int ii = i0 + i;
                const T zg = zgv[i];
                const T cg = fmin(fmax(cw - (T)ii, (T)0), (T)1);
                const T L = Mth<T>::log2((T)1 + zg);
                const T rate = Mth<T>::rcp(Mth<T>::exp2(ra * L) + Mth<T>::exp2(fma(rb, L, rc)));
                vg[ii] = cg * rate * (lp0[i] + fz[i] * (lp1[i] - lp0[i])) * (rec ? Ci : (T)1);
                Ci *= ri;
                ri *= r2;
              }
            }
            if (g0 == 0 && kl == 0) vg[0] *= (T)0.5;
            const T A = Mth<T>::exp2((T)-2 * S * x0l);
            for (int c0 = 0; c0 < n; c0 += 16) {
              T z, w;
              z_w(c0, n, z, w);
              const T zr = (z - (T)ga) * invh;
              const T Bk = Mth<T>::exp2((T)2 * S * zr);
              const int cnt = n - c0 < 16 ? n - c0 : 16;
              if (g0 == 0) {
                const unsigned long long m = __ballot(w > (T)0);
                if (kl == 0 && a.evals)
                  atomicAdd(&work[0], (unsigned long long)__popcll((m >> (16 * q)) & 0xffffull) * a.n_grid);
              }
              T accf[NB];
  #pragma unroll
              for (int i = 0; i < NB; ++i) accf[i] = (T)0;
              int j = 0;
              if (rec) {
                do {
                  const T wj = __shfl(w, j, 16);
                  const T zj = __shfl(zr, j, 16);
                  const T P = A * __shfl(Bk, j, 16);
                  const T x0 = x0l - zj;
                  T u = wj * Mth<T>::exp2(-(x0 * x0));
                  accf[0] += u;
  #pragma unroll
                  for (int i = 1; i < NB; ++i) {
                    u *= P;
                    accf[i] += u;
                  }
                } while (++j < cnt);
              } else {
                do {
                  const T wj = __shfl(w, j, 16);
                  const T zj = __shfl(zr, j, 16);
  #pragma unroll
                  for (int i = 0; i < NB; ++i) {
                    const T xx = fma((T)i, S, x0l) - zj;
                    accf[i] = fma(wj, Mth<T>::exp2(-(xx * xx)), accf[i]);
                  }
                } while (++j < cnt);
              }
              T part = (T)0;
  #pragma unroll
              for (int i = 0; i < NB; ++i) part = fma(vg[i], accf[i], part);
              Tt += (double)part;
            }
          }
          Tt = row_reduce(Tt, [](double x, double y) { return x + y; }) * dz / (hp * 2.5066282746310002);
        }
        if (ract && kl == 0) a.out[((size_t)(tile * GL + lp) * a.n_pix + p) * NF_KDE + 1] = Tt;
      }
    }
  }
  __syncthreads();
  if (a.evals && threadIdx.x < 2 && work[threadIdx.x]) atomicAdd(a.evals + threadIdx.x, work[threadIdx.x]);
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// Per (event, point): merge the event's pixel-part records {R, T, S1, S2} of
// passing pixels (S1 > 0 on a pixel's first part, T > 0 on its others) under
// one exponent.  One wavefront per pair; lanes stride over the parts, then a
// symmetric butterfly.
__global__ __launch_bounds__(256) void kde_event_kernel(const double* __restrict__ pix, const int64_t* ev_part_off,
                                                        int64_t n_parts, int n_events, int B, double* __restrict__ ev) {
  const int lane = threadIdx.x & 63;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= (int64_t)n_events * B) return;
  const int b = (int)(w / n_events), e = (int)(w % n_events);
  int R = R_SENTINEL;
  double T = 0, S1 = 0, S2 = 0;
  for (int64_t p = ev_part_off[e] + lane; p < ev_part_off[e + 1]; p += 64) {
    const double* r = pix + ((size_t)b * n_parts + p) * NF_KDE;
    if (!(r[2] > 0) && !(r[1] > 0)) continue;
    const int Rp = (int)r[0];
    if (R == R_SENTINEL) R = Rp;
    else if (Rp > R) {
      T = ldexp(T, R - Rp);
      S1 = ldexp(S1, R - Rp);
      S2 = ldexp(S2, 2 * (R - Rp));
      R = Rp;
    }
    T += ldexp(r[1], Rp - R);
    S1 += ldexp(r[2], Rp - R);
    S2 += ldexp(r[3], 2 * (Rp - R));
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int Ro = __shfl_xor(R, off);
    const double To = __shfl_xor(T, off), S1o = __shfl_xor(S1, off), S2o = __shfl_xor(S2, off);
    const int Rm = R > Ro ? R : Ro;
    T = ldexp(T, R - Rm) + ldexp(To, Ro - Rm);
    S1 = ldexp(S1, R - Rm) + ldexp(S1o, Ro - Rm);
    S2 = ldexp(S2, 2 * (R - Rm)) + ldexp(S2o, 2 * (Ro - Rm));
    R = Rm;
  }
  if (lane == 0) {
    double* o = ev + ((size_t)b * n_events + e) * NF_KDE;
    o[0] = (double)R;
    o[1] = T;
    o[2] = S1;
    o[3] = S2;
  }
}

// KDE kernel: points per block tile and its dynamic LDS.
template <typename T> struct KdeTile { static constexpr int LT = 64; };
template <> struct KdeTile<double> { static constexpr int LT = 4; };

template <typename T>
static size_t kde_lds_bytes() {
  using T2 = typename V2<T>::t;
  return sizeof(T2) * (size_t)KdeTile<T>::LT * ((Tab<T>::NU + 1) + (Tab<T>::NW + 1));
}

template <typename T, bool SPLIT>
static hipError_t kde_attr() {
  return hipFuncSetAttribute((const void*)kde_kernel<T, KdeTile<T>::LT, SPLIT>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kde_lds_bytes<T>());
}

// Batched kernel: points per tile (the largest the batch fills; FP64 tables
// leave room for four) and its dynamic LDS: per-point tables and constants.
template <typename T, int GL>
static size_t kde_tile_lds_bytes() {
  using T2 = typename V2<T>::t;
  return sizeof(T2) * (size_t)GL * ((Tab<T>::NU + 1) + (Tab<T>::NW + 1)) + sizeof(LamC<T>) * (size_t)GL;
}

template <typename T, int GL>
static hipError_t kde_tile_attr() {
  return hipFuncSetAttribute((const void*)kde_tile_kernel<T, GL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kde_tile_lds_bytes<T, GL>());
}

int kde_tile_points(int fp32, int B) {
  if (!fp32) return 4;
  return B >= 48 ? 64 : (B >= 12 ? 16 : 4);
}

template <typename T, int GL>
static hipError_t kde_tile_t(const KdeArgs& a, int n_cu, hipStream_t st) {
  constexpr int threads = KdeTileThreads<T>::N;
  const int n_tiles = (a.B + GL - 1) / GL;
  const int64_t waves = a.n_pix;   // one task per (pixel, tile)
  int grid_x = (n_cu + n_tiles - 1) / n_tiles;   // one workgroup per CU over the tiles
  if ((int64_t)grid_x * (threads / 64) > waves) grid_x = (int)((waves + threads / 64 - 1) / (threads / 64));
  if (grid_x < 1) grid_x = 1;
  kde_tile_kernel<T, GL><<<dim3(grid_x, n_tiles), threads, kde_tile_lds_bytes<T, GL>(), st>>>(a);
  return hipGetLastError();
}

// Row kernel (fewer than four points): rows take (pixel part, point) pairs.
template <typename T>
static hipError_t kde_t(const KdeArgs& a, int n_cu, hipStream_t st) {
  constexpr int LT = KdeTile<T>::LT;
  const int n_tiles = (a.B + LT - 1) / LT;
  const int64_t tasks = (a.n_parts * a.B + 3) / 4;
  int grid_x = (2 * n_cu + n_tiles - 1) / n_tiles;
  if ((int64_t)grid_x * 8 > tasks) grid_x = (int)((tasks + 7) / 8);
  if (grid_x < 1) grid_x = 1;
  const dim3 grid(grid_x, n_tiles);
  const size_t lds = kde_lds_bytes<T>();
  if (a.parts) kde_kernel<T, LT, true><<<grid, 512, lds, st>>>(a);
  else kde_kernel<T, LT, false><<<grid, 512, lds, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_kde(int fp32, const KdeArgs& a, int n_cu, hipStream_t st) {
  if (a.evals) {
    zero_u64_kernel<<<1, 64, 0, st>>>(a.evals, 2);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.n_parts == 0) return hipSuccess;
  if (a.n_grid < 2 || a.n_grid > KDE_GRID_MAX) return hipErrorInvalidValue;
  if (a.B >= 4 && !a.parts) {   // batched: the tile kernel (whole pixels, records per pixel)
    if (!fp32) return kde_tile_t<double, 4>(a, n_cu, st);
    switch (kde_tile_points(fp32, a.B)) {
      case 64: return kde_tile_t<float, 64>(a, n_cu, st);
      case 16: return kde_tile_t<float, 16>(a, n_cu, st);
      default: return kde_tile_t<float, 4>(a, n_cu, st);
    }
  }
  return fp32 ? kde_t<float>(a, n_cu, st) : kde_t<double>(a, n_cu, st);
}

hipError_t launch_kde_events(const double* pix, const int64_t* ev_part_off, int64_t n_parts, int n_events, int B,
                             double* ev, hipStream_t st) {
  const int64_t threads = (int64_t)n_events * B * 64;
  kde_event_kernel<<<(unsigned)((threads + 255) / 256), 256, 0, st>>>(pix, ev_part_off, n_parts, n_events, B, ev);
  return hipGetLastError();
}

// Raise the dynamic-LDS limit of every KDE variant (once, outside any capture).
hipError_t init_kde_attrs() {
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = kde_attr<float, false>();
  if (e == hipSuccess) e = kde_attr<float, true>();
  if (e == hipSuccess) e = kde_attr<double, false>();
  if (e == hipSuccess) e = kde_attr<double, true>();
  if (e == hipSuccess) e = kde_tile_attr<float, 64>();
  if (e == hipSuccess) e = kde_tile_attr<float, 16>();
  if (e == hipSuccess) e = kde_tile_attr<float, 4>();
  if (e == hipSuccess) e = kde_tile_attr<double, 4>();
  return e;
}

}  // namespace dsl
