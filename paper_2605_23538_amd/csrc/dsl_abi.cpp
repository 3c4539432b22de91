// Host side of the library: catalogue validation and upload, the work list,
// the per-call launch sequence (setup -> sweep -> combine), HIP graph replay,
// options, the autotuner and the extern "C" entry points of include/dsl.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dsl.h"
#include "dsl_internal.h"

namespace dsl {
size_t sweep_lds_bytes(int fp32, int GL, bool grad);
hipError_t launch_pack(int fp32, const double* m1, const double* m2, const double* dl, const double* lnp,
                       int64_t n, void* out, hipStream_t st);
hipError_t launch_setup(int fp32, const double* lam, int B, double z_max, void* lamc, void* cos_tab,
                        void* win_tab, void* win_grad_tab, int* valid, double* gmap, double* unode, int n_z,
                        int32_t* item_ctr, int threads, hipStream_t st);
hipError_t launch_sweep(int fp32, int GL, bool grad, const SweepArgs& a, int grid_x, int threads, hipStream_t st);
hipError_t launch_combine(bool grad, const CombineArgs& a, hipStream_t st);
hipError_t launch_gate_split(const GateSplitArgs& a, hipStream_t st);
hipError_t launch_kde(int fp32, const KdeArgs& a, int n_cu, hipStream_t st);
hipError_t launch_kde_events(const double* pix, const int64_t* ev_part_off, int64_t n_parts, int n_events, int B,
                             double* ev, hipStream_t st);
hipError_t init_kernel_attrs();
hipError_t init_kde_attrs();
}  // namespace dsl

using namespace dsl;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hipfail(hipError_t e, const char* what) {
  return fail(DSL_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) return hipfail(e_, #x);   \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;              // owns its allocation
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  bool fits(size_t bytes) const { return p && bytes <= n; }
  hipError_t ensure(size_t bytes) {
    if (bytes <= n && p) return hipSuccess;
    if (p) {
      (void)hipFree(p);
      p = nullptr;
      n = 0;
    }
    hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
    if (e == hipSuccess) n = bytes;
    return e;
  }
  template <typename X>
  X* as() const {
    return reinterpret_cast<X*>(p);
  }
};

struct SweepCfg {
  int GL = 64;          // Lambda per wavefront
  int64_t chunk = 0;    // target samples per item (0: automatic)
  int waves = 8;        // wavefronts per workgroup
  int wg_per_cu = 2;    // workgroups per CU for the persistent grid
};

struct GraphKey {
  int B;
  bool grad;
  const void* ptrs[8];
  hipStream_t st;
  bool operator<(const GraphKey& o) const {
    if (B != o.B) return B < o.B;
    if (grad != o.grad) return grad < o.grad;
    if (st != o.st) return st < o.st;
    return std::memcmp(ptrs, o.ptrs, sizeof(ptrs)) < 0;
  }
};

}  // namespace

struct dsl_handle {
  int device = 0;
  int fp32 = 1;
  int n_cu = 256;
  int64_t n_events = 0, n_pix = 0, n_samp = 0, n_inj = 0, n_draw = 0, n_rows = 0, n_samp_input = 0;
  int n_z = 0;
  double z_max = 0;
  std::vector<int64_t> epo, pso;   // host copies (work-list builder)
  DevBuf samp, inj, pix_off, pix_row, los, sky, ln_ns;
  // KDE numerator: pixel parts and event -> parts (split grid stage), event ->
  // pixels, per-pixel d_L order
  DevBuf kde_parts, ev_part_off, ev_pix_off, perm, kde_order;
  int64_t n_kde_parts = 0, built_part_size = 0, max_pix_samples = 0;
  int64_t last_kde_units = 0;   // grid-stage units of the last KDE call (pixels or pixel parts)
  // work list (for the current chunk size)
  int64_t built_chunk = -1;
  int built_step = 0;
  DevBuf items, order, ev_item_off, splits;
  int n_items = 0, inj_slot0 = 0, inj_slot1 = 0, n_split = 0;
  // workspace
  DevBuf lamc, cos_tab, win_tab, wg_tab, valid, part, gmap, unode, item_ctr, kde_out, kde_ev, kde_evals, cpart;
  // options
  double neff_min = 2.0;
  int gate_mode = 0;
  int max_batch = 4096;
  int lambda_tile = 0;
  int64_t chunk_opt = 0;
  int timing = 0;
  int graph = 1;
  int z_prior = 0;
  int numerator = 0;         // 0 per-sample Monte Carlo sum, 1 the KDE of Eq. (6)
  int kde_bandwidth = 0;     // 0 Scott, 1 Silverman, 2 biweight (Appendix D)
  int kde_grid = 256;
  int last_gl = 0;           // Lambda tile of the last call
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // setup | sweep | pixels | combine
  bool have_timing = false;
  // recorded after each call's last launch: the host waits on it before it
  // rewrites a device work list, moves a workspace buffer or drops a graph
  // (the caller's stream may be non-blocking, so a synchronous copy on the
  // null stream would not be ordered after that call's kernels)
  hipEvent_t done = nullptr;
  bool pending = false;
  hipStream_t cap_stream = nullptr;
  void* scratch = nullptr;   // device address of the static scratch array on this handle's device
  std::map<GraphKey, hipGraphExec_t> graphs;
  std::vector<const void*> ws_sig;   // workspace addresses the cached graphs were captured with
  std::map<std::pair<int, int>, SweepCfg> tuned;   // (B, grad) -> configuration
  ~dsl_handle() {
    if (pending && done) (void)hipEventSynchronize(done);
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (done) (void)hipEventDestroy(done);
  }
};

// Workspace of the allocation-free entry point (dsl_loglike_grad_noalloc): one
// static device array per GPU, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): it uses the address hipGetSymbolAddress returns, looked up
// once per device with that device current.
constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device ordinal -> device address of `scratch`

// The scratch array's address on `device`, which must be the current device.
int scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail(DSL_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    if (!ptr) return fail(DSL_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    it = g_scratch_ptr.emplace(device, ptr).first;
  }
  *out = it->second;
  return DSL_OK;
}

// Wait until the last call on this handle has finished on the device.
int quiesce(dsl_handle* h) {
  if (h->pending) {
    HIPCHK(hipEventSynchronize(h->done));
    h->pending = false;
  }
  return DSL_OK;
}

void drop_graphs(dsl_handle* h) {
  for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
  h->graphs.clear();
}

bool finite_pos(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!(std::isfinite(a[i]) && a[i] > 0)) return false;
  return true;
}
bool finite_all(const double* a, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

int validate(const dsl_catalog_desc* d) {
  if (!d) return fail(DSL_EINVAL, "desc is NULL");
  if (d->n_events < 1 || !d->event_pix_off) return fail(DSL_EINVAL, "n_events < 1 or event_pix_off NULL");
  // (before any array is read) event and pixel indices are 32-bit on the device
  if (d->n_events >= (int64_t)INT32_MAX) return fail(DSL_EINVAL, "too many events");
  if (d->n_pix >= (int64_t)INT32_MAX) return fail(DSL_EINVAL, "too many pixels");
  if (d->n_pix < 0 || !d->pix_samp_off || (d->n_pix > 0 && !d->pix_los_row))
    return fail(DSL_EINVAL, "pixel arrays missing");
  if (d->n_z < 2 || !(d->z_max > 0) || !std::isfinite(d->z_max)) return fail(DSL_EINVAL, "need n_z >= 2 and z_max > 0");
  // table offsets inside a row are 32-bit byte offsets
  if (d->n_z > (1 << 24)) return fail(DSL_EINVAL, "n_z must be <= 2^24");
  if (d->n_los_rows < 1 || (!d->los == !d->los_f64) || (!d->sky_z == !d->sky_z_f64))
    return fail(DSL_EINVAL, "give exactly one of los / los_f64 and one of sky_z / sky_z_f64");
  if (d->n_samp < 0 || (d->n_samp > 0 && (!d->m1d || !d->m2d || !d->dl || !d->ln_pi)))
    return fail(DSL_EINVAL, "sample arrays missing");
  if (d->n_inj < 1 || !d->inj_m1d || !d->inj_m2d || !d->inj_dl || !d->inj_ln_pdraw)
    return fail(DSL_EINVAL, "need at least one injection");
  if (d->n_draw < d->n_inj) return fail(DSL_EINVAL, "n_draw < n_inj");
  if (d->precision != DSL_PRECISION_FP32 && d->precision != DSL_PRECISION_FP64)
    return fail(DSL_EINVAL, "precision must be 0 (fp64) or 1 (fp32)");
  if (d->event_pix_off[0] != 0 || d->event_pix_off[d->n_events] != d->n_pix)
    return fail(DSL_EINVAL, "event_pix_off must start at 0 and end at n_pix");
  for (int64_t i = 0; i < d->n_events; ++i)
    if (d->event_pix_off[i + 1] < d->event_pix_off[i]) return fail(DSL_EINVAL, "event_pix_off not monotone");
  if (d->pix_samp_off[0] != 0 || d->pix_samp_off[d->n_pix] != d->n_samp)
    return fail(DSL_EINVAL, "pix_samp_off must start at 0 and end at n_samp");
  for (int64_t j = 0; j < d->n_pix; ++j) {
    if (d->pix_samp_off[j + 1] < d->pix_samp_off[j]) return fail(DSL_EINVAL, "pix_samp_off not monotone");
    if (d->pix_los_row[j] < 0 || d->pix_los_row[j] >= d->n_los_rows)
      return fail(DSL_EINVAL, "pix_los_row out of range");
  }
  if (!finite_pos(d->m1d, d->n_samp) || !finite_pos(d->m2d, d->n_samp) || !finite_pos(d->dl, d->n_samp))
    return fail(DSL_EINVAL, "sample masses and distances must be finite and > 0");
  if (!finite_all(d->ln_pi, d->n_samp)) return fail(DSL_EINVAL, "ln_pi must be finite");
  if (!finite_pos(d->inj_m1d, d->n_inj) || !finite_pos(d->inj_m2d, d->n_inj) || !finite_pos(d->inj_dl, d->n_inj))
    return fail(DSL_EINVAL, "injection masses and distances must be finite and > 0");
  if (!finite_all(d->inj_ln_pdraw, d->n_inj)) return fail(DSL_EINVAL, "inj_ln_pdraw must be finite");
  const int64_t nl = d->n_los_rows * (int64_t)d->n_z;
  auto tab_ok = [](const float* f, const double* g, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
      const double v = f ? (double)f[i] : g[i];
      if (!std::isfinite(v) || v < 0) return false;
    }
    return true;
  };
  if (!tab_ok(d->los, d->los_f64, nl)) return fail(DSL_EINVAL, "LOS tables must be finite and >= 0");
  if (!tab_ok(d->sky_z, d->sky_z_f64, d->n_z)) return fail(DSL_EINVAL, "sky_z must be finite and >= 0");
  return DSL_OK;
}

// SplitMix64 (Steele, Lea & Flood 2014): the keys of the per-pixel downsampling.
uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Downsampled {
  dsl_catalog_desc desc;
  std::vector<int64_t> pso;
  std::vector<double> m1, m2, dl, lp;
};

// Keep at most max_samples_per_pixel samples per pixel: those with the
// smallest keys (ties by position), in their original order.
void downsample(const dsl_catalog_desc& d, Downsampled& o) {
  const int64_t cap = d.max_samples_per_pixel;
  o.desc = d;
  o.pso.assign(1, 0);
  std::vector<std::pair<uint64_t, int64_t>> keys;
  std::vector<int64_t> keep;
  for (int64_t j = 0; j < d.n_pix; ++j) {
    const int64_t s0 = d.pix_samp_off[j], n = d.pix_samp_off[j + 1] - s0;
    keep.clear();
    if (n <= cap) {
      for (int64_t k = 0; k < n; ++k) keep.push_back(k);
    } else {
      keys.resize(n);
      for (int64_t k = 0; k < n; ++k)
        keys[k] = {splitmix64(d.downsample_seed + splitmix64(((uint64_t)j << 32) | (uint64_t)k)), k};
      std::nth_element(keys.begin(), keys.begin() + cap, keys.end());
      for (int64_t k = 0; k < cap; ++k) keep.push_back(keys[k].second);
      std::sort(keep.begin(), keep.end());
    }
    for (int64_t k : keep) {
      o.m1.push_back(d.m1d[s0 + k]);
      o.m2.push_back(d.m2d[s0 + k]);
      o.dl.push_back(d.dl[s0 + k]);
      o.lp.push_back(d.ln_pi[s0 + k]);
    }
    o.pso.push_back((int64_t)o.m1.size());
  }
  o.desc.pix_samp_off = o.pso.data();
  o.desc.n_samp = (int64_t)o.m1.size();
  o.desc.m1d = o.m1.data();
  o.desc.m2d = o.m2.data();
  o.desc.dl = o.dl.data();
  o.desc.ln_pi = o.lp.data();
}

int upload(DevBuf& b, const void* src, size_t bytes) {
  hipError_t e = b.ensure(bytes);
  if (e != hipSuccess) return fail(DSL_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  if (bytes && src) HIPCHK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
  return DSL_OK;
}

// Redshift-prior tables in the handle's precision (float32 for FP32 handles,
// float64 for FP64 ones) from float32 or float64 input; a conversion goes
// through a host staging slice, so a 10 GB catalogue needs no second copy.
int upload_table(dsl_handle* h, DevBuf& b, const float* f32, const double* f64, int64_t n) {
  const size_t el = h->fp32 ? sizeof(float) : sizeof(double);
  if ((h->fp32 && f32) || (!h->fp32 && f64)) return upload(b, f32 ? (const void*)f32 : (const void*)f64, el * n);
  int rc = upload(b, nullptr, el * (size_t)n);
  if (rc) return rc;
  const int64_t slice = 1 << 22;
  std::vector<float> sf(h->fp32 ? (size_t)std::min(n, slice) : 0);
  std::vector<double> sd(h->fp32 ? 0 : (size_t)std::min(n, slice));
  for (int64_t i0 = 0; i0 < n; i0 += slice) {
    const int64_t m = std::min(slice, n - i0);
    if (h->fp32) {
      for (int64_t i = 0; i < m; ++i) sf[i] = (float)f64[i0 + i];
      HIPCHK(hipMemcpy(b.as<float>() + i0, sf.data(), sizeof(float) * m, hipMemcpyHostToDevice));
    } else {
      for (int64_t i = 0; i < m; ++i) sd[i] = (double)f32[i0 + i];
      HIPCHK(hipMemcpy(b.as<double>() + i0, sd.data(), sizeof(double) * m, hipMemcpyHostToDevice));
    }
  }
  return DSL_OK;
}

int pack_samples(dsl_handle* h, DevBuf& out, const double* m1, const double* m2, const double* dl,
                 const double* lnp, int64_t n) {
  const size_t rec = h->fp32 ? sizeof(Samp<float>) : sizeof(Samp<double>);
  hipError_t e = out.ensure(rec * (size_t)std::max<int64_t>(n, 1));
  if (e != hipSuccess) return fail(DSL_ENOMEM, std::string("hipMalloc samples: ") + hipGetErrorString(e));
  // stream the raw arrays through a staging buffer in slices
  const int64_t slice = 1 << 22;
  DevBuf stage;
  e = stage.ensure(4 * sizeof(double) * (size_t)std::min<int64_t>(std::max<int64_t>(n, 1), slice));
  if (e != hipSuccess) return fail(DSL_ENOMEM, "hipMalloc staging");
  for (int64_t s = 0; s < n; s += slice) {
    const int64_t m = std::min(slice, n - s);
    double* st = stage.as<double>();
    HIPCHK(hipMemcpy(st, m1 + s, m * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(st + m, m2 + s, m * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(st + 2 * m, dl + s, m * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(st + 3 * m, lnp + s, m * sizeof(double), hipMemcpyHostToDevice));
    char* dst = out.as<char>() + rec * (size_t)s;
    HIPCHK(launch_pack(h->fp32, st, st + m, st + 2 * m, st + 3 * m, m, dst, nullptr));
    HIPCHK(hipDeviceSynchronize());
  }
  return DSL_OK;
}

// Default work-item size: about 256 items per compute unit for batched tiles
// and 64 for one-point tiles, at least 256 samples for batched tiles (each
// item writes one record per point, which the combine reads back) and 64 for
// one-point tiles.
int64_t auto_chunk(const dsl_handle* h, int GL) {
  const int64_t total = h->n_samp + h->n_inj;
  const int64_t per_cu = GL == 1 ? 64 : 256;
  const int64_t lo = GL == 1 ? 64 : 256;
  int64_t c = total / ((int64_t)h->n_cu * per_cu);
  return std::max<int64_t>(lo, std::min<int64_t>(16384, c));
}

// Work list: runs of whole pixels of one event (about `chunk` samples each; a
// larger pixel forms its own item) and runs of `chunk` injections.  A pixel
// counts as its sample count rounded up to `step`: with one point per
// wavefront (step 64) a pixel of 3 samples takes as long as one of 64, so a
// run of many small pixels would otherwise become the launch's long tail
// (one-point sweep of the 140-event catalogue: 106 -> 75 us per call).  With
// several points per wavefront the rounding moved nothing but the item count
// (+2.5 %), so there step is 1.  Slots are in event order; the processing
// order puts the largest items first.
int build_items(dsl_handle* h, int64_t chunk, int step) {
  if (chunk == h->built_chunk && step == h->built_step) return DSL_OK;
  int rc0 = quiesce(h);   // the previous call may still read the current list
  if (rc0) return rc0;
  std::vector<WorkItem> it;
  std::vector<SplitPix> sp;
  std::vector<int32_t> ev_off(h->n_events + 1, 0);
  // pixels with more than 2 chunks of samples are split into parts of one chunk
  const int64_t split_thr = 2 * chunk;
  for (int64_t e = 0; e < h->n_events; ++e) {
    ev_off[e] = (int32_t)it.size();
    const int64_t p0 = h->epo[e], p1 = h->epo[e + 1];
    int64_t a = p0;
    while (a < p1) {
      if (h->pso[a + 1] - h->pso[a] > split_thr) {
        SplitPix s;
        s.slot0 = (int32_t)it.size();
        s.n_parts = 0;
        for (int64_t x = h->pso[a]; x < h->pso[a + 1]; x += chunk) {
          WorkItem w;
          w.event = (int32_t)e;
          w.pix0 = w.pix1 = (int32_t)a;
          w.slot = (int32_t)it.size();
          w.s0 = x;
          w.s1 = std::min(h->pso[a + 1], x + chunk);
          it.push_back(w);
          ++s.n_parts;
        }
        sp.push_back(s);
        ++a;
        continue;
      }
      auto cost = [&](int64_t q) { return (h->pso[q + 1] - h->pso[q] + step - 1) / step * step; };
      int64_t b = a + 1;
      int64_t n = cost(a);
      while (b < p1 && n + cost(b) <= chunk && h->pso[b + 1] - h->pso[b] <= split_thr) {
        n += cost(b);
        ++b;
      }
      WorkItem w;
      w.event = (int32_t)e;
      w.pix0 = (int32_t)a;
      w.pix1 = (int32_t)b;
      w.slot = (int32_t)it.size();
      w.s0 = h->pso[a];
      w.s1 = h->pso[b];
      it.push_back(w);
      a = b;
    }
  }
  ev_off[h->n_events] = (int32_t)it.size();
  const int inj0 = (int)it.size();
  for (int64_t s = 0; s < h->n_inj; s += chunk) {
    WorkItem w;
    w.event = -1;
    w.pix0 = w.pix1 = 0;
    w.slot = (int32_t)it.size();
    w.s0 = s;
    w.s1 = std::min(h->n_inj, s + chunk);
    it.push_back(w);
  }
  if (it.size() >= (size_t)INT32_MAX) return fail(DSL_EINVAL, "work list too long: use a larger chunk");
  std::vector<int32_t> ord(it.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int32_t)i;
  auto cost = [&](int32_t i) {
    int64_t c = 0;
    if (it[i].event < 0 || it[i].pix1 == it[i].pix0) c = (it[i].s1 - it[i].s0 + step - 1) / step * step;
    else
      for (int64_t q = it[i].pix0; q < it[i].pix1; ++q) c += (h->pso[q + 1] - h->pso[q] + step - 1) / step * step;
    return c + 4 * (int64_t)(it[i].pix1 - it[i].pix0);
  };
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return cost(x) > cost(y); });
  int rc;
  if ((rc = upload(h->items, it.data(), it.size() * sizeof(WorkItem)))) return rc;
  if ((rc = upload(h->order, ord.data(), ord.size() * sizeof(int32_t)))) return rc;
  if ((rc = upload(h->ev_item_off, ev_off.data(), ev_off.size() * sizeof(int32_t)))) return rc;
  if (sp.empty()) {
    if (h->splits.ensure(sizeof(SplitPix)) != hipSuccess) return fail(DSL_ENOMEM, "hipMalloc splits");
  } else if ((rc = upload(h->splits, sp.data(), sp.size() * sizeof(SplitPix)))) {
    return rc;
  }
  h->n_split = (int)sp.size();
  h->n_items = (int)it.size();
  h->inj_slot0 = inj0;
  h->inj_slot1 = (int)it.size();
  h->built_chunk = chunk;
  h->built_step = step;
  drop_graphs(h);
  return DSL_OK;
}

// Default Lambda tile: the largest the batch fills (64 from 48 points, 16 from
// 12, 4 from 3) that still leaves at least 128 work units (item x tile) per
// compute unit; small catalogues take narrow tiles so that every CU has work.
int default_gl(const dsl_handle* h, int B) {
  if (!h->fp32) return B >= 4 ? 4 : 1;
  const int cap = B >= 48 ? 64 : (B >= 12 ? 16 : (B >= 3 ? 4 : 1));
  const int64_t total = h->n_samp + h->n_inj;
  for (int gl = cap; gl > 4; gl /= 4) {
    const int64_t chunk = auto_chunk(h, gl);
    const int64_t units = ((total + chunk - 1) / chunk) * ((B + gl - 1) / gl);
    if (units >= 128 * (int64_t)h->n_cu) return gl;
  }
  return cap < 4 ? cap : 4;
}

// Workgroup shape of the sweep. The FP32 adjoint fits 3 waves per SIMD (<= 168
// VGPRs): 64-point tiles take 117 KB of LDS, so one 12-wavefront workgroup per
// CU; smaller tiles three 4-wavefront workgroups. Shape 1 is the plain 8 x 2.
void block_shape(const dsl_handle* h, bool grad, int GL, int shape, SweepCfg& c) {
  if (h->fp32 && grad && shape == 0) {
    c.waves = GL == 64 ? 12 : 4;
    c.wg_per_cu = GL == 64 ? 1 : 3;
  } else if (h->fp32 && !grad && shape == 2) {
    // the FP32 forward sweep of one point fits 6 waves per SIMD (<= 84 VGPRs):
    // three 8-wavefront workgroups per CU hide more of the table-gather latency
    c.waves = 8;
    c.wg_per_cu = 3;
  } else {
    c.waves = 8;
    c.wg_per_cu = 2;
  }
}

SweepCfg config_for(dsl_handle* h, int B, bool grad) {
  auto it = h->tuned.find({B, grad ? 1 : 0});
  SweepCfg c;
  if (it != h->tuned.end()) c = it->second;
  else c.GL = default_gl(h, B);
  if (h->lambda_tile) c.GL = h->lambda_tile;
  if (!h->fp32 && c.GL > 4) c.GL = 4;
  if (h->chunk_opt) c.chunk = h->chunk_opt;
  if (c.chunk <= 0) c.chunk = auto_chunk(h, c.GL);
  if (it == h->tuned.end() || h->lambda_tile) block_shape(h, grad, c.GL, h->fp32 && !grad && c.GL == 1 ? 2 : 0, c);
  return c;
}

// Combine workgroups per point: about one per 256 work items, at most 32, and
// no more than 8 per compute unit over the batch.
int combine_slices(const dsl_handle* h, int B) {
  const int by_items = (h->n_items + 255) / 256;
  const int by_cu = (8 * h->n_cu + B - 1) / B;
  return std::max(1, std::min(32, std::min(by_items, by_cu)));
}

// Part size of the KDE grid stage for fewer than four points (the row kernel):
// a pixel holding more than half the samples a wavefront handles on average
// over the launch would be a long tail, so pixels above max(KDE_PART, that
// half) are split into parts of that many samples (a multiple of 16).  0: no
// pixel is split.
int64_t kde_part_size(const dsl_handle* h, int B) {
  if (B >= 4) return 0;   // batches take the tile kernel, which walks whole pixels largest first
  const double per_wave = (double)h->n_samp * B / (4.0 * 16 * h->n_cu);
  int64_t P = std::max<int64_t>(KDE_PART, (int64_t)std::ceil(0.5 * per_wave));
  P = (P + 15) / 16 * 16;
  return h->max_pix_samples > P ? P : 0;
}

// The part list for part size P (rebuilt when P changes; graphs read it at
// replay, and a reallocation drops them through the workspace signature).
int build_kde_parts(dsl_handle* h, int64_t P) {
  if (P == 0 || P == h->built_part_size) return DSL_OK;
  int rc0 = quiesce(h);
  if (rc0) return rc0;
  std::vector<KdePart> parts;
  std::vector<int64_t> ev_part(h->n_events + 1);
  for (int64_t e = 0; e < h->n_events; ++e) {
    ev_part[e] = (int64_t)parts.size();
    for (int64_t j = h->epo[e]; j < h->epo[e + 1]; ++j) {
      const int64_t n = h->pso[j + 1] - h->pso[j];
      int64_t lo = 0;
      do {
        KdePart pt;
        pt.pix = j;
        pt.lo = (int32_t)lo;
        pt.hi = (int32_t)std::min<int64_t>(n, lo + P);
        parts.push_back(pt);
        lo += P;
      } while (lo < n);
    }
  }
  ev_part[h->n_events] = (int64_t)parts.size();
  int rc;
  if ((rc = upload(h->kde_parts, parts.data(), sizeof(KdePart) * parts.size()))) return rc;
  if ((rc = upload(h->ev_part_off, ev_part.data(), sizeof(int64_t) * ev_part.size()))) return rc;
  h->n_kde_parts = (int64_t)parts.size();
  h->built_part_size = P;
  return DSL_OK;
}

// Events spanning many work items (the monte-carlo numerator) are merged by one
// wavefront of the combine each, instead of one thread walking the items.
bool merge_events(const dsl_handle* h) {
  return h->numerator == 0 && h->n_events > 0 && h->inj_slot0 >= 16 * h->n_events;
}

// Device workspace of one call: the handle's buffers, or (for the
// allocation-free entry point) ranges of the per-device static scratch.
struct Ws {
  void* lamc = nullptr;
  void* cos_tab = nullptr;
  void* win_tab = nullptr;
  void* wg_tab = nullptr;
  void* valid = nullptr;
  void* gmap = nullptr;
  void* unode = nullptr;   // FP64 (1+z) I(z) at the table nodes (FP32 adjoint)
  void* item_ctr = nullptr;   // per-tile work-item counters, per-point slice counters
  void* part = nullptr;
  void* cpart = nullptr;
  void* kde_out = nullptr;
  void* kde_ev = nullptr;
  void* kde_evals = nullptr;
};

// The workspace buffers of a call with B points: the handle's buffer, the
// field of `ws` it fills, and its size.
struct WsNeed {
  DevBuf* buf;
  void** dst;
  size_t bytes;
  const char* what;
};

struct WsNeeds {
  WsNeed v[15];
  int n = 0;
  void add(DevBuf* b, void** d, size_t bytes, const char* what) { v[n++] = WsNeed{b, d, bytes, what}; }
  const WsNeed* begin() const { return v; }
  const WsNeed* end() const { return v + n; }
};

WsNeeds workspace_needs(dsl_handle* h, int B, bool grad, Ws& ws) {
  const int NU = h->fp32 ? NU_F32 : NU_F64, NW = h->fp32 ? NW_F32 : NW_F64;
  const int NWG = h->fp32 ? NWG_F32 : NWG_F64;
  const size_t t1 = h->fp32 ? sizeof(float) : sizeof(double);
  const size_t lc = h->fp32 ? sizeof(LamC<float>) : sizeof(LamC<double>);
  const size_t nf = grad ? NF_GRAD : NF_FWD;
  const size_t Bz = (size_t)B;
  WsNeeds n;
  n.add(&h->lamc, &ws.lamc, lc * Bz, "lamc");
  n.add(&h->cos_tab, &ws.cos_tab, 2 * t1 * (NU + 1) * Bz, "cos");
  n.add(&h->win_tab, &ws.win_tab, 2 * t1 * (NW + 1) * Bz, "win");
  n.add(&h->wg_tab, &ws.wg_tab, 6 * t1 * (NWG + 1) * Bz, "wg");
  n.add(&h->valid, &ws.valid, sizeof(int) * Bz, "valid");
  n.add(&h->gmap, &ws.gmap, sizeof(double) * N_GMAP * Bz, "gmap");
  if (h->fp32 && grad) n.add(&h->unode, &ws.unode, sizeof(double) * (size_t)h->n_z * Bz, "FP64 node values");
  n.add(&h->item_ctr, &ws.item_ctr, 3 * sizeof(int32_t) * Bz, "work-item and slice counters");
  n.add(&h->part, &ws.part, sizeof(double) * nf * Bz * (size_t)std::max(h->n_items, 1), "partials");
  n.add(&h->cpart, &ws.cpart, sizeof(double) * NF_CSLICE * Bz * (size_t)combine_slices(h, B), "combine slices");
  if (h->numerator == 1) {
    const int64_t units = std::max<int64_t>(kde_part_size(h, B) ? h->n_kde_parts : h->n_pix, 1);
    n.add(&h->kde_out, &ws.kde_out, sizeof(double) * NF_KDE * Bz * (size_t)units, "KDE pixel terms");
    n.add(&h->kde_evals, &ws.kde_evals, 2 * sizeof(unsigned long long), "KDE counter");
    n.add(&h->kde_ev, &ws.kde_ev, sizeof(double) * NF_KDE * Bz * (size_t)std::max<int64_t>(h->n_events, 1),
          "KDE event terms");
  }
  return n;
}

// The handle's workspace for B points, grown when needed.
int ensure_workspace(dsl_handle* h, int B, bool grad, Ws& ws) {
  const WsNeeds need = workspace_needs(h, B, grad, ws);
  bool grow = false;
  for (const WsNeed& w : need) grow = grow || !w.buf->fits(w.bytes);
  if (grow) {   // a buffer moves: the previous call must be done with it
    const int rc = quiesce(h);
    if (rc) return rc;
  }
  for (const WsNeed& w : need) {
    if (w.buf->ensure(w.bytes) != hipSuccess) return fail(DSL_ENOMEM, std::string("workspace (") + w.what + ")");
    *w.dst = w.buf->p;
  }
  return DSL_OK;
}

struct CallOut {
  double* logL;
  double* grad;
  double* logL_event;
  double* neff_event;
  double* neff_sel;
  uint32_t* flags;
};

// Enqueue setup -> sweep -> combine on st (no synchronisation).
int enqueue(dsl_handle* h, const Ws& ws, const double* d_lambda, int B, bool grad, const CallOut& o,
            const SweepCfg& cfg, hipStream_t st, bool timed) {
  if (timed) HIPCHK(hipEventRecord(h->ev[0], st));
  // setup: two workgroups per point; wide ones shorten a call when they leave CUs free
  const int setup_threads = 2 * B < h->n_cu ? 1024 : 256;
  HIPCHK(launch_setup(h->fp32, d_lambda, B, h->z_max, ws.lamc, ws.cos_tab, ws.win_tab,
                      grad ? ws.wg_tab : nullptr, (int*)ws.valid, grad ? (double*)ws.gmap : nullptr,
                      (double*)ws.unode, h->n_z, (int32_t*)ws.item_ctr, setup_threads, st));
  if (timed) HIPCHK(hipEventRecord(h->ev[1], st));
  SweepArgs a;
  a.samp = h->samp.p;
  a.inj = h->inj.p;
  a.pix_off = h->pix_off.as<int64_t>();
  a.pix_row = h->pix_row.as<int32_t>();
  a.los = h->los.p;
  a.sky = h->sky.p;
  a.n_z = h->n_z;
  a.z_max = h->z_max;
  a.unode = (const double*)ws.unode;
  // batched tiles take work items from a counter (dealt by a fixed stride the
  // largest-first list loads some workgroups with the largest item of every
  // round); one point per wavefront keeps the stride: its many small items
  // would contend on the one counter
  a.item_ctr = cfg.GL > 1 ? (int32_t*)ws.item_ctr : nullptr;
  a.items = h->items.as<WorkItem>();
  a.order = h->order.as<int32_t>();
  a.n_items = h->n_items;
  a.lamc = ws.lamc;
  a.cos_tab = ws.cos_tab;
  a.win_tab = ws.win_tab;
  a.win_grad_tab = ws.wg_tab;
  a.B = B;
  a.neff_min = h->neff_min;
  a.gate_mode = h->gate_mode;
  a.z_prior = h->z_prior;
  a.skip_events = h->numerator == 1;
  a.part = (double*)ws.part;
  const int n_tiles = (B + cfg.GL - 1) / cfg.GL;
  const int waves = cfg.waves;
  int grid_x = std::max(1, (h->n_cu * cfg.wg_per_cu + n_tiles - 1) / n_tiles);
  grid_x = std::min(grid_x, std::max(1, (h->n_items + waves - 1) / waves));
  HIPCHK(launch_sweep(h->fp32, cfg.GL, grad, a, grid_x, 64 * waves, st));
  if (timed) HIPCHK(hipEventRecord(h->ev[4], st));
  GateSplitArgs gs;
  gs.part = (double*)ws.part;
  gs.n_items = h->n_items;
  gs.nf = grad ? NF_GRAD : NF_FWD;
  gs.B = B;
  gs.splits = h->splits.as<SplitPix>();
  gs.n_split = h->n_split;
  gs.neff_min = h->neff_min;
  gs.gate_mode = h->gate_mode;
  if (h->numerator == 1) {
    KdeArgs k;
    k.samp = h->samp.p;
    k.pix_off = h->pix_off.as<int64_t>();
    k.pix_row = h->pix_row.as<int32_t>();
    k.perm = h->perm.as<int32_t>();
    k.los = h->los.p;
    k.n_z = h->n_z;
    k.z_max = h->z_max;
    k.n_pix = h->n_pix;
    k.order = h->kde_order.as<int32_t>();
    const bool split = kde_part_size(h, B) != 0;   // part list built for this B before the launch
    k.parts = split ? h->kde_parts.as<KdePart>() : nullptr;
    k.n_parts = split ? h->n_kde_parts : h->n_pix;
    h->last_kde_units = k.n_parts;
    k.lamc = ws.lamc;
    k.cos_tab = ws.cos_tab;
    k.win_tab = ws.win_tab;
    k.B = B;
    k.bandwidth = h->kde_bandwidth;
    k.n_grid = h->kde_grid;
    k.tau = 5.0;
    k.neff_min = h->neff_min;
    k.gate_mode = h->gate_mode;
    k.out = (double*)ws.kde_out;
    k.evals = (unsigned long long*)ws.kde_evals;
    k.pix_ctr = (int32_t*)ws.item_ctr + B;
    HIPCHK(launch_kde(h->fp32, k, h->n_cu, st));
    HIPCHK(launch_kde_events((const double*)ws.kde_out, split ? h->ev_part_off.as<int64_t>() : h->ev_pix_off.as<int64_t>(),
                             k.n_parts, (int)h->n_events, B,
                             (double*)ws.kde_ev, st));
  } else {
    HIPCHK(launch_gate_split(gs, st));
  }
  if (timed) HIPCHK(hipEventRecord(h->ev[2], st));
  CombineArgs c;
  c.part = (const double*)ws.part;
  c.n_items = h->n_items;
  c.nf = grad ? NF_GRAD : NF_FWD;
  c.B = B;
  c.n_events = (int32_t)h->n_events;
  c.ev_item_off = h->ev_item_off.as<int32_t>();
  c.inj_slot0 = h->inj_slot0;
  c.inj_slot1 = h->inj_slot1;
  c.ln_ns = h->ln_ns.as<double>();
  c.ln_ndraw = std::log((double)h->n_draw);
  c.neff_min = h->neff_min;
  c.gate_mode = h->gate_mode;
  c.valid = (const int*)ws.valid;
  c.logL = o.logL;
  c.logL_event = o.logL_event;
  c.neff_event = o.neff_event;
  c.neff_sel = o.neff_sel;
  c.flags = o.flags;
  c.grad = o.grad;
  c.gmap = (const double*)ws.gmap;
  c.kde = h->numerator == 1 ? (const double*)ws.kde_ev : nullptr;
  c.wave_events = merge_events(h) ? 1 : 0;
  c.n_slices = combine_slices(h, B);
  c.cpart = (double*)ws.cpart;
  // The last slice to finish merges the others only in small grids: each slice
  // orders its record before its count with a device-scope fence, which on
  // this multi-die part includes an L2 write-back (64 points x 32 slices:
  // combine 0.23 -> 0.29 ms with the fences; one point: 13.2 -> 11.1 us for
  // the event merge, combine and slice merge together).
  c.slice_ctr = B * c.n_slices <= 64 ? (int32_t*)ws.item_ctr + 2 * B : nullptr;
  HIPCHK(launch_combine(grad, c, st));
  if (timed) HIPCHK(hipEventRecord(h->ev[3], st));
  return DSL_OK;
}

int run(dsl_handle* h, const double* d_lambda, int B, bool grad, const CallOut& o, hipStream_t st) {
  if (!h) return fail(DSL_ESTATE, "handle is NULL");
  (void)hipGetLastError();   // the launch checks below must not see an earlier call's error
  if (!d_lambda || !o.logL || (grad && !o.grad)) return fail(DSL_EINVAL, "NULL device pointer");
  if (B < 1 || B > h->max_batch) return fail(DSL_EINVAL, "B out of range [1, max_batch]");
  if (h->numerator == 1 && grad) return fail(DSL_EINVAL, "the KDE numerator has no gradient (use numerator 0)");
  if (h->numerator == 1 && h->z_prior != 0)
    return fail(DSL_EINVAL, "the KDE numerator needs the LOS redshift tables (z_prior 0)");
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != h->device) return fail(DSL_ESTATE, "current device differs from the handle's device");
  const SweepCfg cfg = config_for(h, B, grad);
  h->last_gl = cfg.GL;
  int rc;
  if ((rc = build_items(h, cfg.chunk, cfg.GL == 1 ? 64 : 1))) return rc;
  if (h->numerator == 1 && (rc = build_kde_parts(h, kde_part_size(h, B)))) return rc;
  Ws ws;
  if ((rc = ensure_workspace(h, B, grad, ws))) return rc;
  // captured graphs hold workspace addresses: drop them all when any buffer moved
  const std::vector<const void*> sig = {h->items.p,   h->order.p,   h->ev_item_off.p, h->splits.p, h->lamc.p,
                                        h->cos_tab.p, h->win_tab.p, h->wg_tab.p,      h->valid.p,  h->gmap.p,
                                        h->unode.p,   h->item_ctr.p,
                                        h->part.p,    h->kde_out.p, h->kde_ev.p,      h->kde_evals.p, h->cpart.p,
                                        h->kde_parts.p, h->ev_part_off.p};
  if (sig != h->ws_sig) {   // (a buffer that moved waited for the previous call first)
    drop_graphs(h);
    h->ws_sig = sig;
  }
  if (h->timing) {
    h->have_timing = true;
    rc = enqueue(h, ws, d_lambda, B, grad, o, cfg, st, true);
  } else if (!h->graph) {
    rc = enqueue(h, ws, d_lambda, B, grad, o, cfg, st, false);
  } else {
    GraphKey k{};
    k.B = B;
    k.grad = grad;
    k.st = st;
    const void* ptrs[8] = {d_lambda, o.logL, o.grad, o.logL_event, o.neff_event, o.neff_sel, o.flags,
                           (const void*)(intptr_t)(((cfg.GL * 1000003 + cfg.chunk) * 64 + cfg.waves) * 8 + cfg.wg_per_cu)};
    std::memcpy(k.ptrs, ptrs, sizeof(ptrs));
    auto it = h->graphs.find(k);
    if (it == h->graphs.end()) {
      if (h->graphs.size() >= 16) {
        if ((rc = quiesce(h))) return rc;
        drop_graphs(h);
      }
      HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
      rc = enqueue(h, ws, d_lambda, B, grad, o, cfg, h->cap_stream, false);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return hipfail(e, "hipStreamEndCapture");
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hipfail(e, "hipGraphInstantiate");
      it = h->graphs.emplace(k, ex).first;
    }
    const hipError_t e = hipGraphLaunch(it->second, st);
    rc = e == hipSuccess ? DSL_OK : hipfail(e, "hipGraphLaunch");
  }
  // marks the end of this call's work on st, also after a failed launch
  // (whatever was enqueued before the failure must finish before the next rewrite)
  const hipError_t er = hipEventRecord(h->done, st);
  if (er == hipSuccess) h->pending = true;
  if (rc) return rc;
  return er == hipSuccess ? DSL_OK : hipfail(er, "hipEventRecord");
}

// The allocation-free variant of run() (gradient entry point): the workspace is
// carved out of the device's static scratch array; the work list in place is
// used whatever chunk it was built for (the chunk only sets how the sums are
// cut into items); no graph, no timing events, no host-to-device copy.
int run_noalloc(dsl_handle* h, const double* d_lambda, int B, const CallOut& o, hipStream_t st) {
  if (!h) return fail(DSL_ESTATE, "handle is NULL");
  (void)hipGetLastError();
  if (!d_lambda || !o.logL || !o.grad) return fail(DSL_EINVAL, "NULL device pointer");
  if (B < 1 || B > h->max_batch) return fail(DSL_EINVAL, "B out of range [1, max_batch]");
  if (h->numerator == 1) return fail(DSL_EINVAL, "the KDE numerator has no gradient (use numerator 0)");
  int cur = -1;
  HIPCHK(hipGetDevice(&cur));
  if (cur != h->device) return fail(DSL_ESTATE, "current device differs from the handle's device");
  if (!h->scratch || h->built_chunk < 0) return fail(DSL_ESTATE, "handle has no scratch address or work list");
  SweepCfg cfg = config_for(h, B, true);
  cfg.chunk = h->built_chunk;
  h->last_gl = cfg.GL;
  Ws ws;
  const WsNeeds need = workspace_needs(h, B, true, ws);
  size_t off = 0;
  for (const WsNeed& w : need) {
    off = (off + 255) & ~(size_t)255;
    if (w.bytes > SCRATCH_BYTES || off + w.bytes > SCRATCH_BYTES)
      return fail(DSL_EINVAL, "this batch needs more than the " + std::to_string(SCRATCH_BYTES >> 20) +
                                  " MiB scratch of the allocation-free entry point (use dsl_loglike_grad)");
    *w.dst = static_cast<unsigned char*>(h->scratch) + off;
    off += w.bytes;
  }
  const int rc = enqueue(h, ws, d_lambda, B, true, o, cfg, st, false);
  // a later call that rewrites the work list waits for this one
  const hipError_t er = hipEventRecord(h->done, st);
  if (er == hipSuccess) h->pending = true;
  if (rc) return rc;
  return er == hipSuccess ? DSL_OK : hipfail(er, "hipEventRecord");
}

// Sweep configurations the autotuner may choose for batches of B points:
// Lambda tiles (a tile is skipped when it would leave most lanes idle), chunks
// about the automatic size, and for the FP32 adjoint both workgroup shapes.
std::vector<SweepCfg> tune_candidates(const dsl_handle* h, int B, bool grad) {
  std::vector<SweepCfg> out;
  const std::vector<int> gls = h->fp32 ? std::vector<int>{1, 4, 16, 64} : std::vector<int>{1, 4};
  for (int gl : gls) {
    if (gl > 1 && B < gl / 4) continue;
    const int64_t base = auto_chunk(h, gl);
    std::vector<int64_t> chunks;
    for (int64_t ch : {base / 16, base / 4, base, base * 4}) {
      ch = std::max<int64_t>(64, std::min<int64_t>(65536, ch));
      if (std::find(chunks.begin(), chunks.end(), ch) == chunks.end()) chunks.push_back(ch);
    }
    // workgroup shapes: both FP32-adjoint shapes; for forward one-point tiles
    // also three workgroups per CU
    std::vector<int> shapes{0};
    if (h->fp32 && grad) shapes.push_back(1);
    if (h->fp32 && !grad && gl == 1) shapes.push_back(2);
    for (int shape : shapes)
      for (int64_t ch : chunks) {
        SweepCfg c;
        c.GL = gl;
        c.chunk = ch;
        block_shape(h, grad, gl, shape, c);
        out.push_back(c);
      }
  }
  return out;
}

// A cached entry is taken only if its tile and workgroup shape are ones this
// library launches and its chunk lies in the range the tuner explores.
bool cached_cfg_ok(const dsl_handle* h, bool grad, const SweepCfg& c) {
  if (c.chunk < 64 || c.chunk > 65536) return false;
  if (!(c.GL == 1 || c.GL == 4 || (h->fp32 && (c.GL == 16 || c.GL == 64)))) return false;
  for (int shape = 0; shape < 3; ++shape) {
    SweepCfg s;
    block_shape(h, grad, c.GL, shape, s);
    if (s.waves == c.waves && s.wg_per_cu == c.wg_per_cu) return true;
  }
  return false;
}

// Times every candidate (one warm-up call, then three) and returns the fastest
// in `best`.  The caller restores the handle's options.
int tune_sweep(dsl_handle* h, int B, bool grad, SweepCfg& best) {
  // scratch Lambda batch: the prior's centre replicated (valid everywhere)
  std::vector<double> lam(16 * (size_t)B);
  const double centre[16] = {70, 0.3, 2.9, 1.0, 4.6, 86.3, 4.8, 9.7, 0.7, 30.7, 6.3, 0.4, 0.8, 3.3, 2.9, 2.5};
  for (int b = 0; b < B; ++b)
    for (int p = 0; p < 16; ++p) lam[16 * b + p] = centre[p];
  DevBuf dl, dout, dg;
  if (dl.ensure(sizeof(double) * 16 * B) || dout.ensure(sizeof(double) * B) || dg.ensure(sizeof(double) * 16 * B))
    return fail(DSL_ENOMEM, "autotune scratch");
  HIPCHK(hipMemcpy(dl.p, lam.data(), sizeof(double) * 16 * B, hipMemcpyHostToDevice));
  struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } ev;
  HIPCHK(hipEventCreate(&ev.e0));
  HIPCHK(hipEventCreate(&ev.e1));
  const std::pair<int, int> slot{B, grad ? 1 : 0};
  CallOut o{dout.as<double>(), grad ? dg.as<double>() : nullptr, nullptr, nullptr, nullptr, nullptr};
  double best_ms = 1e300;
  for (const SweepCfg& c : tune_candidates(h, B, grad)) {
    h->tuned[slot] = c;
    int rc = run(h, dl.as<double>(), B, grad, o, nullptr);   // warm-up (and workspace)
    if (rc) return rc;
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipEventRecord(ev.e0, nullptr));
    const int reps = 3;
    for (int r = 0; r < reps; ++r)
      if ((rc = run(h, dl.as<double>(), B, grad, o, nullptr))) return rc;
    HIPCHK(hipEventRecord(ev.e1, nullptr));
    HIPCHK(hipEventSynchronize(ev.e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ev.e0, ev.e1));
    if (ms / reps < best_ms) {
      best_ms = ms / reps;
      best = c;
    }
  }
  return best_ms < 1e300 ? DSL_OK : fail(DSL_ESTATE, "autotune found no candidate");
}

}  // namespace

extern "C" {

const char* dsl_last_error(void) { return g_err.c_str(); }

const char* dsl_version(void) { return "dsl 0.1 (gfx950)"; }

int dsl_create(const dsl_catalog_desc* d_in, dsl_handle** out) {
  if (!out) return fail(DSL_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(d_in);
  if (rc) return rc;
  if (d_in->max_samples_per_pixel < 0) return fail(DSL_EINVAL, "max_samples_per_pixel must be >= 0");
  Downsampled ds;
  const dsl_catalog_desc* d = d_in;
  if (d_in->max_samples_per_pixel > 0) {
    downsample(*d_in, ds);
    d = &ds.desc;
  }
  std::unique_ptr<dsl_handle> h(new (std::nothrow) dsl_handle());
  if (!h) return fail(DSL_ENOMEM, "host allocation");
  (void)hipGetLastError();
  HIPCHK(hipGetDevice(&h->device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, h->device));
  h->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  h->fp32 = d->precision == DSL_PRECISION_FP32;
  h->n_events = d->n_events;
  h->n_pix = d->n_pix;
  h->n_samp = d->n_samp;
  h->n_samp_input = d_in->n_samp;
  h->n_inj = d->n_inj;
  h->n_draw = d->n_draw;
  h->n_rows = d->n_los_rows;
  h->n_z = d->n_z;
  h->z_max = d->z_max;
  h->epo.assign(d->event_pix_off, d->event_pix_off + d->n_events + 1);
  h->pso.assign(d->pix_samp_off, d->pix_samp_off + d->n_pix + 1);
  std::vector<double> ln_ns(d->n_events);
  for (int64_t e = 0; e < d->n_events; ++e) {
    const int64_t ns = h->pso[h->epo[e + 1]] - h->pso[h->epo[e]];
    ln_ns[e] = ns > 0 ? std::log((double)ns) : 0.0;
  }
  if ((rc = upload(h->pix_off, d->pix_samp_off, sizeof(int64_t) * (d->n_pix + 1)))) return rc;
  if ((rc = upload(h->pix_row, d->pix_los_row, sizeof(int32_t) * std::max<int64_t>(d->n_pix, 1)))) return rc;
  if ((rc = upload_table(h.get(), h->los, d->los, d->los_f64, d->n_los_rows * (int64_t)d->n_z))) return rc;
  if ((rc = upload_table(h.get(), h->sky, d->sky_z, d->sky_z_f64, d->n_z))) return rc;
  if ((rc = upload(h->ln_ns, ln_ns.data(), sizeof(double) * ln_ns.size()))) return rc;
  for (int64_t j = 0; j < d->n_pix; ++j) h->max_pix_samples = std::max(h->max_pix_samples, h->pso[j + 1] - h->pso[j]);
  if ((rc = upload(h->ev_pix_off, d->event_pix_off, sizeof(int64_t) * (d->n_events + 1)))) return rc;
  {
    // per pixel, local sample indices in ascending d_L (ties by position): the
    // order of the samples' redshifts for every point, used by the KDE bandwidths
    std::vector<int32_t> perm(std::max<int64_t>(d->n_samp, 1));
    for (int64_t j = 0; j < d->n_pix; ++j) {
      const int64_t a = h->pso[j], n = h->pso[j + 1] - a;
      int32_t* q = perm.data() + a;
      for (int64_t k = 0; k < n; ++k) q[k] = (int32_t)k;
      const double* x = d->dl + a;
      std::sort(q, q + n, [x](int32_t u, int32_t v) { return x[u] < x[v] || (x[u] == x[v] && u < v); });
    }
    if ((rc = upload(h->perm, perm.data(), sizeof(int32_t) * d->n_samp))) return rc;
    // pixels by decreasing sample count (ties by index): the batched KDE kernel's
    // task order, so the largest pixels start first
    std::vector<int32_t> ord(std::max<int64_t>(d->n_pix, 1));
    for (int64_t j = 0; j < d->n_pix; ++j) ord[j] = (int32_t)j;
    std::stable_sort(ord.begin(), ord.begin() + d->n_pix, [&](int32_t u, int32_t v) {
      return h->pso[u + 1] - h->pso[u] > h->pso[v + 1] - h->pso[v];
    });
    if ((rc = upload(h->kde_order, ord.data(), sizeof(int32_t) * ord.size()))) return rc;
  }
  if ((rc = pack_samples(h.get(), h->samp, d->m1d, d->m2d, d->dl, d->ln_pi, d->n_samp))) return rc;
  if ((rc = pack_samples(h.get(), h->inj, d->inj_m1d, d->inj_m2d, d->inj_dl, d->inj_ln_pdraw, d->n_inj))) return rc;
  for (auto& e : h->ev) HIPCHK(hipEventCreate(&e));
  HIPCHK(hipEventCreateWithFlags(&h->done, hipEventDisableTiming));
  HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  HIPCHK(init_kernel_attrs());
  HIPCHK(init_kde_attrs());
  if ((rc = scratch_address(h->device, &h->scratch))) return rc;
  // a work list from the start (the one-point configuration's), so that the
  // allocation-free entry point always has one to read
  const SweepCfg one = config_for(h.get(), 1, false);
  if ((rc = build_items(h.get(), one.chunk, one.GL == 1 ? 64 : 1))) return rc;
  *out = h.release();
  return DSL_OK;
}

void dsl_destroy(dsl_handle* h) { delete h; }

int dsl_set_option(dsl_handle* h, const char* key, double v) {
  if (!h) return fail(DSL_ESTATE, "handle is NULL");
  if (!key) return fail(DSL_EINVAL, "key is NULL");
  const std::string k(key);
  if (!std::isfinite(v)) return fail(DSL_EINVAL, "value must be finite");
  if (k == "neff_min") {
    if (v < 0) return fail(DSL_EINVAL, "neff_min must be >= 0");
    h->neff_min = v;
  } else if (k == "gate_mode") {
    if (v != 0 && v != 1 && v != 2) return fail(DSL_EINVAL, "gate_mode must be 0, 1 or 2");
    h->gate_mode = (int)v;
  } else if (k == "max_batch") {
    if (v < 1 || v > (1 << 20)) return fail(DSL_EINVAL, "max_batch out of range");
    h->max_batch = (int)v;
  } else if (k == "lambda_tile") {
    const int g = (int)v;
    if (v != g || !(g == 0 || g == 1 || g == 4 || g == 16 || g == 64)) return fail(DSL_EINVAL, "lambda_tile must be 0, 1, 4, 16 or 64");
    if (!h->fp32 && g > 4) return fail(DSL_EINVAL, "fp64 supports lambda_tile 0, 1 or 4");
    h->lambda_tile = g;
  } else if (k == "chunk") {
    if (v < 0 || v > (1 << 24)) return fail(DSL_EINVAL, "chunk out of range");
    h->chunk_opt = (int64_t)v;
  } else if (k == "z_prior") {
    if (v != 0 && v != 1) return fail(DSL_EINVAL, "z_prior must be 0 (LOS tables) or 1 (comoving volume)");
    h->z_prior = (int)v;
  } else if (k == "numerator") {
    if (v != 0 && v != 1) return fail(DSL_EINVAL, "numerator must be 0 (per-sample sum) or 1 (KDE)");
    h->numerator = (int)v;
  } else if (k == "kde_bandwidth") {
    if (v != 0 && v != 1 && v != 2) return fail(DSL_EINVAL, "kde_bandwidth must be 0 (Scott), 1 (Silverman) or 2 (biweight)");
    h->kde_bandwidth = (int)v;
  } else if (k == "kde_grid") {
    if (v != (int)v || v < 2 || v > KDE_GRID_MAX) return fail(DSL_EINVAL, "kde_grid must be an integer in [2, 1024]");
    h->kde_grid = (int)v;
  } else if (k == "timing") {
    h->timing = v != 0;
  } else if (k == "graph") {
    h->graph = v != 0;
  } else {
    return fail(DSL_EINVAL, "unknown option '" + k + "'");
  }
  // graphs bake in option values (and may still be running)
  const int rc = quiesce(h);
  if (rc) return rc;
  drop_graphs(h);
  return DSL_OK;
}

int dsl_get_info(dsl_handle* h, const char* key, double* v) {
  if (!h) return fail(DSL_ESTATE, "handle is NULL");
  if (!key || !v) return fail(DSL_EINVAL, "NULL argument");
  const std::string k(key);
  if (k == "n_events") *v = (double)h->n_events;
  else if (k == "n_pix") *v = (double)h->n_pix;
  else if (k == "n_samp") *v = (double)h->n_samp;
  else if (k == "n_samp_input") *v = (double)h->n_samp_input;
  else if (k == "n_inj") *v = (double)h->n_inj;
  else if (k == "n_draw") *v = (double)h->n_draw;
  else if (k == "n_z") *v = (double)h->n_z;
  else if (k == "n_items") *v = (double)h->n_items;
  else if (k == "n_split") *v = (double)h->n_split;
  else if (k == "precision") *v = h->fp32 ? DSL_PRECISION_FP32 : DSL_PRECISION_FP64;
  else if (k == "neff_min") *v = h->neff_min;
  else if (k == "gate_mode") *v = h->gate_mode;
  else if (k == "z_prior") *v = h->z_prior;
  else if (k == "numerator") *v = h->numerator;
  else if (k == "kde_bandwidth") *v = h->kde_bandwidth;
  else if (k == "kde_grid") *v = h->kde_grid;
  else if (k == "max_batch") *v = h->max_batch;
  else if (k == "lambda_tile") *v = h->lambda_tile;
  else if (k == "graph") *v = h->graph;
  else if (k == "timing") *v = h->timing;
  else if (k == "chunk") *v = (double)(h->chunk_opt ? h->chunk_opt : h->built_chunk);
  else if (k == "n_cu") *v = h->n_cu;
  else if (k == "lambda_tile_used") *v = h->last_gl;
  else if (k == "kde_units") *v = (double)h->last_kde_units;
  else if (k == "kde_evals" || k == "kde_nodes") {
    // of the last KDE call (waits for the device): (sample, grid node) kernel
    // terms, and grid nodes (each a prior and rate evaluation) over all
    // (pixel, point) pairs with a bandwidth > 0
    if (!h->kde_evals.p) return fail(DSL_ESTATE, "no KDE call yet");
    unsigned long long n[2] = {0, 0};
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(n, h->kde_evals.p, sizeof(n), hipMemcpyDeviceToHost));
    *v = (double)n[k == "kde_nodes" ? 1 : 0];
  } else if (k == "ms_sweep_only" || k == "ms_pixels") {
    // of the last timed call: the sweep alone, and the per-pixel stage after it
    // (KDE kernel, or the gate of split pixels)
    if (!h->have_timing) return fail(DSL_ESTATE, "no timed call yet (set option 'timing' to 1)");
    HIPCHK(hipEventSynchronize(h->ev[3]));
    float ms = 0;
    if (k == "ms_sweep_only") HIPCHK(hipEventElapsedTime(&ms, h->ev[1], h->ev[4]));
    else HIPCHK(hipEventElapsedTime(&ms, h->ev[4], h->ev[2]));
    *v = ms;
  }
  else if (k == "work_list_bytes") *v = (double)(h->items.n + h->order.n + h->ev_item_off.n + h->splits.n);
  else if (k == "device_bytes") {
    const DevBuf* bufs[] = {&h->samp,      &h->inj,      &h->pix_off,    &h->pix_row,   &h->los,   &h->sky,
                            &h->ln_ns,     &h->kde_parts, &h->ev_part_off, &h->ev_pix_off, &h->perm, &h->kde_order,
                            &h->items,
                            &h->order,     &h->ev_item_off, &h->splits,  &h->lamc,      &h->cos_tab, &h->win_tab,
                            &h->wg_tab,    &h->valid,    &h->part,       &h->gmap,      &h->unode, &h->item_ctr, &h->kde_out, &h->kde_ev,
                            &h->kde_evals, &h->cpart};
    double sum = 0;
    for (const DevBuf* b : bufs) sum += (double)b->n;
    *v = sum;
  } else return fail(DSL_EINVAL, "unknown info key '" + k + "'");
  return DSL_OK;
}

int dsl_loglike(dsl_handle* h, const double* d_lambda, int B, double* d_logL, double* d_logL_event,
                double* d_neff_event, double* d_neff_sel, uint32_t* d_flags, void* stream) {
  CallOut o{d_logL, nullptr, d_logL_event, d_neff_event, d_neff_sel, d_flags};
  return run(h, d_lambda, B, false, o, (hipStream_t)stream);
}

int dsl_loglike_grad(dsl_handle* h, const double* d_lambda, int B, double* d_logL, double* d_grad,
                     double* d_logL_event, double* d_neff_event, double* d_neff_sel, uint32_t* d_flags,
                     void* stream) {
  CallOut o{d_logL, d_grad, d_logL_event, d_neff_event, d_neff_sel, d_flags};
  return run(h, d_lambda, B, true, o, (hipStream_t)stream);
}

int dsl_loglike_grad_noalloc(dsl_handle* h, const double* d_lambda, int B, double* d_logL, double* d_grad,
                             double* d_logL_event, double* d_neff_event, double* d_neff_sel, uint32_t* d_flags,
                             void* stream) {
  CallOut o{d_logL, d_grad, d_logL_event, d_neff_event, d_neff_sel, d_flags};
  return run_noalloc(h, d_lambda, B, o, (hipStream_t)stream);
}

int dsl_get_timing(dsl_handle* h, float* ms_setup, float* ms_sweep, float* ms_combine) {
  if (!h) return fail(DSL_ESTATE, "handle is NULL");
  if (!h->have_timing) return fail(DSL_ESTATE, "no timed call yet (set option 'timing' to 1)");
  HIPCHK(hipEventSynchronize(h->ev[3]));
  float a = 0, b = 0, c = 0;
  HIPCHK(hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
  HIPCHK(hipEventElapsedTime(&b, h->ev[1], h->ev[2]));
  HIPCHK(hipEventElapsedTime(&c, h->ev[2], h->ev[3]));
  if (ms_setup) *ms_setup = a;
  if (ms_sweep) *ms_sweep = b;
  if (ms_combine) *ms_combine = c;
  return DSL_OK;
}

int dsl_autotune(dsl_handle* h, int B, int with_grad, const char* cache_path) {
  if (!h) return fail(DSL_ESTATE, "handle is NULL");
  if (B < 1 || B > h->max_batch) return fail(DSL_EINVAL, "B out of range");
  const bool grad = with_grad != 0;
  char devname[64] = {0};
  {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, h->device));
    std::snprintf(devname, sizeof(devname), "%s", prop.gcnArchName);
  }
  // everything the sweep's cost depends on, without spaces
  std::ostringstream keyss;
  keyss << devname << "|fp32=" << h->fp32 << "|grad=" << grad << "|B=" << B << "|samp=" << h->n_samp
        << "|inj=" << h->n_inj << "|pix=" << h->n_pix << "|ev=" << h->n_events << "|zprior=" << h->z_prior
        << "|num=" << h->numerator;
  std::string key = keyss.str();
  std::replace(key.begin(), key.end(), ' ', '_');
  const std::pair<int, int> slot{B, grad ? 1 : 0};
  // cache lookup: one line per entry, "key GL chunk waves wg_per_cu"
  if (cache_path) {
    std::ifstream f(cache_path);
    std::string line;
    while (std::getline(f, line)) {
      std::istringstream ls(line);
      std::string k;
      SweepCfg c;
      if (ls >> k >> c.GL >> c.chunk >> c.waves >> c.wg_per_cu && k == key && cached_cfg_ok(h, grad, c)) {
        h->tuned[slot] = c;
        return DSL_OK;
      }
    }
  }
  const int saved_tile = h->lambda_tile, saved_graph = h->graph, saved_timing = h->timing;
  const int64_t saved_chunk = h->chunk_opt;
  h->lambda_tile = 0;
  h->chunk_opt = 0;
  h->graph = 0;
  h->timing = 0;
  SweepCfg best;
  const int rc = tune_sweep(h, B, grad, best);
  h->lambda_tile = saved_tile;
  h->chunk_opt = saved_chunk;
  h->graph = saved_graph;
  h->timing = saved_timing;
  if (rc) {
    h->tuned.erase(slot);
    return rc;
  }
  h->tuned[slot] = best;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    f << key << " " << best.GL << " " << best.chunk << " " << best.waves << " " << best.wg_per_cu << "\n";
    if (!f) return fail(DSL_EINVAL, "cannot append to the autotune cache file");
  }
  return DSL_OK;
}

}  // extern "C"
