// Plan objects and the C ABI (include/dks_poisson.h): argument validation,
// radix plans of the three transforms, workspace layout, and the launch
// sequences of the plan-time Green's spectrum and of each solve.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dks_internal.h"
#include "fft_engine.h"
#include "fft_plan_check.h"

namespace dks {

// Launchers defined in the kernel translation units.
template <typename T> hipError_t launch_fft_x_fwd(const void*, size_t, void*, size_t, const MeshDims&,
                                                  const PlanRef&, const void*, int, hipStream_t);
template <typename T> hipError_t launch_fft_y_fwd(const void*, void*, size_t, const MeshDims&, const PlanRef&, int, int,
                                                  int, hipStream_t);
template <typename T> hipError_t launch_fft_z_conv(const void*, void*, size_t, const void*, const Geometry*,
                                                   size_t, const MeshDims&, const PlanRef&, const PlanRef&, int,
                                                   int, int, hipStream_t);
template <typename T> hipError_t launch_fft_y_inv(const void*, void*, size_t, const MeshDims&, const PlanRef&,
                                                  int, int, int, hipStream_t);
template <typename T> hipError_t launch_fft_x_inv(const void*, size_t, void*, size_t, const ElemBatch&,
                                                  const MeshDims&, const PlanRef&, const void*, int,
                                                  hipStream_t);
hipError_t launch_store_plans(const FFTPlan* four, FFTPlan* dev, hipStream_t s);
template <typename T> hipError_t launch_bbox(const ElemBatch&, int, double*, size_t, int*, hipStream_t);
hipError_t launch_geometry(const double*, size_t, Geometry*, size_t, const GeoArgs&, const ElemBatch&, int,
                           hipStream_t);
hipError_t launch_geometry_zero(const double*, size_t, Geometry*, size_t, const GeoArgs&, const ElemBatch&, int,
                                void*, size_t, size_t, hipStream_t);
template <typename T> hipError_t launch_weights_to_density(const void*, void*, size_t, const Geometry*, double,
                                                           hipStream_t);
template <typename T> hipError_t launch_gradient(const void*, void*, const Geometry*, const MeshDims&, hipStream_t);
template <typename T> hipError_t launch_gather(const void*, const void*, const void*, const void*, void*, void*,
                                               void*, int64_t, const Geometry*, const MeshDims&, int, hipStream_t);
template <typename T> hipError_t launch_bin_count(const ElemBatch&, int, const Geometry*, size_t, char*, size_t,
                                                  const MeshDims&, const BinGeom&, int, hipStream_t);
hipError_t launch_bin_scan(const Geometry*, size_t, char*, size_t, const BinGeom&, const ElemBatch&, int,
                           hipStream_t);
template <typename T> hipError_t launch_bin_scatter(const ElemBatch&, int, const Geometry*, size_t, char*,
                                                    size_t, char*, size_t, size_t, const MeshDims&, const BinGeom&,
                                                    int, void* const*, hipStream_t);
template <typename T> hipError_t launch_deposit_binned(const Geometry*, size_t, char*, size_t, const char*, size_t,
                                                       void*, size_t, const MeshDims&, const BinGeom&, int, int, void* const*,
                                                       void*, size_t, hipStream_t);
template <typename T> hipError_t launch_fixed_to_weights(const void*, size_t, void*, size_t, size_t, int, hipStream_t);
template <typename T> hipError_t launch_gather_binned(const Geometry*, size_t, char*, size_t, char*, size_t,
                                                      const void*, size_t, const MeshDims&, const BinGeom&, int, int,
                                                      void* const*, hipStream_t);
template <typename T> hipError_t launch_unsort(const ElemBatch&, int, const char*, size_t, size_t, hipStream_t);
template <typename T> hipError_t launch_twiddle_pass(void*, int, int, hipStream_t);
template <typename T> hipError_t launch_twiddle_line(void*, int, int, hipStream_t);
hipError_t launch_igf_octant(double*, const int*, const double*, const GLBands&, int, hipStream_t);
hipError_t launch_cos_matrix(double*, int, hipStream_t);
hipError_t launch_apply_axis(const double*, double*, const double*, const int*, int, hipStream_t);
template <typename T> hipError_t launch_green_pack(const double*, void*, const int*, int, int, double, hipStream_t);

static inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Particles per solve: binned positions are 32-bit, and a lane's loop index
// may run up to 2^20 past the end of its range before the bound check.
constexpr int64_t kMaxParticles = (int64_t(1) << 32) - (int64_t(1) << 20);

static bool factor23(int N) {
  if (N < 1) return false;
  while (N % 2 == 0) N /= 2;
  while (N % 3 == 0) N /= 3;
  return N == 1;
}

// Radix-8 passes first, then one radix-4 or radix-2 pass for the remaining
// powers of two, then radix-3 passes; pass 0 is even whenever N is.
static std::vector<int> radices_for(int N) {
  int a = 0, b = 0;
  while (N % 2 == 0) { N /= 2; ++a; }
  while (N % 3 == 0) { N /= 3; ++b; }
  std::vector<int> r;
  while (a >= 3) { r.push_back(8); a -= 3; }
  if (a == 2) r.push_back(4);
  if (a == 1) r.push_back(2);
  for (int i = 0; i < b; ++i) r.push_back(3);
  return r;
}

static int pick_width(int N, size_t csize, bool padded, int wmax) {
  int W = wmax;
  while (W > 1 && (size_t)N * (size_t)(padded ? W + 1 : W) * csize > (size_t)kLdsBytes) W >>= 1;
  return W;
}

static void build_fft(FFTPlanHost& P, int N, const std::vector<int>& R, int W, bool padded) {
  std::memset(&P, 0, sizeof(P));
  P.dev.N = N;
  P.dev.npass = (int)R.size();
  P.dev.W = W;
  int lw = 0;
  while ((1 << lw) < W) ++lw;
  P.dev.logW = lw;
  P.dev.LD = padded ? W + 1 : W;
  int Ns = 1, off = 0;
  for (size_t p = 0; p < R.size(); ++p) {
    P.dev.R[p] = R[p];
    P.dev.Ns[p] = Ns;
    P.dev.magic[p] = Ns >= 2 ? (unsigned)(((1ull << 32) + (unsigned long long)Ns - 1) / (unsigned long long)Ns) : 0u;
    P.dev.tw_off[p] = off;
    if (p > 0) off += Ns * (R[p] - 1);
    Ns *= R[p];
  }
  P.tw_count = off;
}

// Nodes and weights of the m-point Gauss-Legendre rule on [-1, 1] (Newton
// iteration on the three-term Legendre recurrence).
static void gauss_legendre(int m, double* x, double* w) {
  for (int i = 0; i < m; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= m; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = m * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= m; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = m * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

static GLBands make_bands() {
  GLBands g;
  std::memset(&g, 0, sizeof(g));
  const double lo[5] = {2.0, 4.0, 8.0, 16.0, 32.0};
  const int m[5] = {10, 8, 6, 5, 4};
  g.nb = 5;
  for (int i = 0; i < 5; ++i) {
    g.lo[i] = lo[i];
    g.m[i] = m[i];
    gauss_legendre(m[i], g.t[i], g.w[i]);
  }
  return g;
}

}  // namespace dks

using namespace dks;

// State of host-resident solves.  Two staging slots hold a solve's device
// copy of rho and of its outputs; solve k uses slot k % 2.  Uploads and
// downloads run on two copy streams of the plan, the kernels on the caller's
// stream; the events order the three.  Downloads are issued in ticket order
// on one stream, so they land in ticket order.
constexpr int kHostRing = 8;
struct HostPipe {
  char* stage;
  size_t stage_bytes;
  int device;                     // device of the streams; -1 before the first solve
  hipStream_t up, down;           // copy streams (default priority, non-blocking)
  hipEvent_t computed[2];         // slot's kernels done: input read, outputs written
  hipEvent_t uploaded[2];         // slot's input on the device
  hipEvent_t landed[kHostRing];   // ticket's outputs on the host
  uint64_t issued;                // tickets handed out so far
};

struct dks_poisson_plan_s {
  int n[3];
  double h[3];
  double origin[3];
  bool fitted;
  dks_dtype dtype;
  int green;        // dks_green: kernel of the convolution
  size_t rsize;     // sizeof(real)
  size_t csize;     // sizeof(complex)
  MeshDims md;
  FFTPlanHost px, py, pz, pzi;
  size_t off_plans;                                        // four device FFTPlan copies
  size_t tw_px, tw_py, tw_pz, tw_pzi, tw_post, tw_bytes;   // byte offsets in the twiddle region
  size_t off_green, green_bytes, off_slot;
  // slot layout (bytes from slot start)
  size_t s_bbox, s_bins, s_r1, s_r2, s_r3, slot_bytes;
  size_t bytes_W, bytes_phi_ext;
  BinGeom bg;          // tiles of the binned deposit/gather (item set per solve)
  int bins_len;        // uint32 entries of the bin bookkeeping
  size_t part_elem;    // bytes per binned particle record (x, y, z; later the field)
  size_t ws_total;
  char* ws;
  size_t ws_bytes;
  char* pscratch;      // caller-owned binned-particle scratch of single solves
  size_t pscratch_bytes;
  bool prepared;
  bool has_geometry;
  bool deterministic = false;   // order-independent deposit (integer node totals)
  HostPipe hp;         // host-resident solves
};

namespace {

dks_status hip_status(hipError_t e) { return e == hipSuccess ? DKS_OK : DKS_EHIP; }

// Particle scratch of np particles: the binned records, then the inverse
// permutation (uint32 per particle).
size_t inv_offset(const dks_poisson_plan_s* p, int64_t np) { return align256((size_t)np * p->part_elem); }
size_t particle_bytes(const dks_poisson_plan_s* p, int64_t np) {
  return inv_offset(p, np) + align256((size_t)np * sizeof(unsigned));
}

// Optional per-kernel event timing (dks_timing_enable / dks_timing_read).
struct TimingState {
  std::mutex mu;
  bool on = false;
  struct Rec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void release_all() {
    for (auto& r : recs) {
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
};

TimingState& timing() {
  static TimingState t;
  return t;
}

// Records an event before the launch and one after it, when timing is on.
class Timed {
 public:
  Timed(const char* name, hipStream_t st) : name_(name), st_(st) {
    TimingState& t = timing();
    std::lock_guard<std::mutex> lock(t.mu);
    if (!t.on) return;
    a_ = t.take();
    if (a_ && hipEventRecord(a_, st_) == hipSuccess) active_ = true;
  }
  void done() {
    if (!active_) return;
    TimingState& t = timing();
    std::lock_guard<std::mutex> lock(t.mu);
    hipEvent_t b = t.take();
    if (b && hipEventRecord(b, st_) == hipSuccess) t.recs.push_back({name_, a_, b});
    active_ = false;
  }

 private:
  const char* name_;
  hipStream_t st_;
  hipEvent_t a_ = nullptr;
  bool active_ = false;
};

#define DKS_CK(call)                              \
  do {                                            \
    const hipError_t e_ = (call);                 \
    if (e_ != hipSuccess) return DKS_EHIP;        \
  } while (0)

// Launch `call` on stream `st` under the kernel name `name` for the timing records.
#define DKS_TK(name, call)                        \
  do {                                            \
    Timed tm_(name, st);                          \
    const hipError_t e_ = (call);                 \
    if (e_ != hipSuccess) return DKS_EHIP;        \
    tm_.done();                                   \
  } while (0)

// The pass kernels' limits for the dtype (what fft_engine.h is built with).
template <typename T> EngineLimits engine_limits() {
  EngineLimits L;
  L.threads = RegCfg<T>::THREADS;
  L.emax = RegCfg<T>::EMAX;
  L.max_length = kMaxLength;
  L.max_pass = kMaxPass;
  L.lds_hw = kLdsHardware;
  return L;
}

// Checks the four plans against the invariants of the pass kernels that use
// them: x forward (rows of nx reals staged through kTileReals registers per
// thread, nx + 1 post-twiddles in LDS beside the tile), x inverse (rows of N
// complex values staged the same way), y, z forward and z inverse (pencils
// read straight from memory).  Returns the first violation, or kPlanOk.
int check_plans(const dks_poisson_plan_s* p) {
  const EngineLimits L = p->dtype == DKS_F32 ? engine_limits<float>() : engine_limits<double>();
  const size_t c = p->csize;
  const int nx = p->md.nx;
  int v = fft_plan_violation(p->px.dev, L, c, nx, kTileReals, (size_t)(nx + 1) * c);
  if (v == kPlanOk) v = fft_plan_violation(p->px.dev, L, c, p->px.dev.N, kTileReals, 0);
  if (v == kPlanOk) v = fft_plan_violation(p->py.dev, L, c, 0, 0, 0);
  if (v == kPlanOk) v = fft_plan_violation(p->pz.dev, L, c, 0, 0, 0);
  if (v == kPlanOk) v = fft_plan_violation(p->pzi.dev, L, c, 0, 0, 0);
  return v;
}

void layout(dks_poisson_plan_s* p) {
  const int nx = p->n[0], ny = p->n[1], nz = p->n[2];
  const size_t s = p->rsize, c = p->csize;
  const int wmax = (int)(128 / c);    // 128-byte column tiles
  MeshDims& m = p->md;
  m.nx = nx; m.ny = ny; m.nz = nz;
  m.Nx = 2 * nx; m.Ny = 2 * ny; m.Nz = 2 * nz;
  m.ncols = nx + 1;
  m.cs = (nx + 1 + wmax - 1) / wmax * wmax;
  const int Wx = pick_width(nx, c, true, wmax);
  const int Wy = pick_width(m.Ny, c, false, wmax);
  const int Wz = pick_width(m.Nz, c, false, wmax);
  build_fft(p->px, nx, radices_for(nx), Wx, true);
  build_fft(p->py, m.Ny, radices_for(m.Ny), Wy, false);
  std::vector<int> rz = radices_for(m.Nz);
  build_fft(p->pz, m.Nz, rz, Wz, false);
  std::reverse(rz.begin(), rz.end());
  build_fft(p->pzi, m.Nz, rz, Wz, false);
  size_t off = 0;
  p->off_plans = off; off = align256(off + 4 * sizeof(FFTPlan));
  p->tw_px = off; off = align256(off + p->px.tw_count * c);
  p->tw_py = off; off = align256(off + p->py.tw_count * c);
  p->tw_pz = off; off = align256(off + p->pz.tw_count * c);
  p->tw_pzi = off; off = align256(off + p->pzi.tw_count * c);
  p->tw_post = off; off = align256(off + (size_t)(nx + 1) * c);
  p->tw_bytes = off;
  p->off_green = off;
  p->green_bytes = (size_t)(ny + 1) * (nz + 1) * m.cs * s;
  p->off_slot = align256(p->off_green + p->green_bytes);
  const size_t cs = (size_t)m.cs;
  const size_t A = (size_t)ny * nz * cs * c;
  // B and C are block-major: (2 ny) rows of cs columns over nz (B) or nz + 2 (C) planes
  const size_t B = (size_t)m.Ny * nz * cs * c;
  const size_t C = (size_t)m.Ny * (nz + 2) * cs * c;
  const size_t D = (size_t)(ny + 2) * (nz + 2) * cs * c;
  p->bytes_W = (size_t)nx * ny * nz * s;
  p->bytes_phi_ext = (size_t)(nx + 2) * (ny + 2) * (nz + 2) * s;
  const size_t G64 = (size_t)(nx + 1) * (ny + 1) * (nz + 1) * sizeof(double);
  const size_t COS = ((size_t)(nx + 1) * (nx + 1) + (size_t)(ny + 1) * (ny + 1) + (size_t)(nz + 1) * (nz + 1)) *
                     sizeof(double);
  const size_t r1 = std::max({A, C, G64});
  // R2 also holds the order-independent deposit's integer node totals (8 or
  // 16 bytes per node; B alone always covers them)
  const size_t r2 = std::max({B, D, G64, (size_t)nx * ny * nz * 2 * s});
  const size_t r3 = std::max({p->bytes_W, p->bytes_phi_ext, COS + 256});
  BinGeom& bg = p->bg;
  bg.tx = (nx + 15) / 16;        // 16 nodes per tile edge (CIC files by cell, NGP/TSC by node)
  bg.ty = (ny + 15) / 16;
  bg.tz = (nz + 15) / 16;
  bg.K = bg.tx * bg.ty * bg.tz;
  bg.item = 65536;
  bg.lds_hist = 2 * (size_t)(bg.K + 1) * sizeof(unsigned) <= 65536 ? 1 : 0;
  p->bins_len = bins_entries(bg.K);
  p->part_elem = 3 * s;
  size_t so = align256(sizeof(Geometry));
  p->s_bbox = so; so = align256(so + (size_t)kBboxBlocks * 6 * sizeof(double));
  p->s_bins = so; so = align256(so + (size_t)p->bins_len * sizeof(unsigned));
  p->s_r1 = so; so = align256(so + r1);
  p->s_r2 = so; so = align256(so + r2);
  p->s_r3 = so; so = align256(so + r3);
  p->slot_bytes = so;
  p->ws_total = p->off_slot + p->slot_bytes;
}

// idx: 0 = x, 1 = y, 2 = z forward, 3 = z inverse.
PlanRef planref(const dks_poisson_plan_s* p, int idx) {
  const FFTPlanHost* hs[4] = {&p->px, &p->py, &p->pz, &p->pzi};
  const size_t offs[4] = {p->tw_px, p->tw_py, p->tw_pz, p->tw_pzi};
  PlanRef r;
  r.host = hs[idx]->dev;
  r.host.tw = p->ws + offs[idx];
  r.dev = reinterpret_cast<const FFTPlan*>(p->ws + p->off_plans) + idx;
  return r;
}

struct Slots {
  char* base;
  size_t stride;   // bytes between consecutive elements
  Geometry* geo() const { return reinterpret_cast<Geometry*>(base); }
};

// rho (in `src`, element stride in_stride) -> phi_ext in R3 (+ user phi) via the five passes.
template <typename T>
dks_status convolve(const dks_poisson_plan_s* p, const void* src, size_t in_stride, int batch, const Slots& sl,
                    const ElemBatch& phi_user, hipStream_t st) {
  const MeshDims& m = p->md;
  const size_t cstride = sl.stride / p->csize;
  const size_t rstride = sl.stride / p->rsize;
  char* R1 = sl.base + p->s_r1;
  char* R2 = sl.base + p->s_r2;
  char* R3 = sl.base + p->s_r3;
  const PlanRef fx = planref(p, 0);
  const PlanRef fy = planref(p, 1);
  const PlanRef fz = planref(p, 2);
  const PlanRef fzi = planref(p, 3);
  const void* post = p->ws + p->tw_post;
  const void* G = p->ws + p->off_green;
  DKS_TK("fft_x_fwd", launch_fft_x_fwd<T>(src, in_stride, R1, cstride, m, fx, post, batch, st));
  DKS_TK("fft_y_fwd", launch_fft_y_fwd<T>(R1, R2, cstride, m, fy, batch, 0, m.ncols, st));
  DKS_TK("fft_z_conv", launch_fft_z_conv<T>(R2, R1, cstride, G, sl.geo(), sl.stride, m, fz, fzi, batch, 0, m.ncols, st));
  DKS_TK("fft_y_inv", launch_fft_y_inv<T>(R1, R2, cstride, m, fy, batch, 0, m.ncols, st));
  DKS_TK("fft_x_inv", launch_fft_x_inv<T>(R2, cstride, R3, rstride, phi_user, m, fx, post, batch, st));
  return DKS_OK;
}

GeoArgs geo_args(const dks_poisson_plan_s* p, int mode, int nblocks) {
  GeoArgs a;
  std::memset(&a, 0, sizeof(a));
  for (int d = 0; d < 3; ++d) {
    a.n[d] = p->n[d];
    a.h[d] = p->h[d];
    a.origin[d] = p->origin[d];
  }
  a.fitted = p->fitted ? 1 : 0;
  a.nblocks = nblocks;
  a.mode = mode;
  a.zero_off = 0;
  a.zero_len = 0;
  return a;
}

// Work split of one (batched) particle solve.
struct PartWork {
  BinGeom bg;
  int count_blocks;   // blocks of the count and scatter kernels (same chunking)
  int item_blocks;    // blocks of the deposit and gather kernels (loop over work items)
};

PartWork part_work(const dks_poisson_plan_s* p, int64_t maxn) {
  PartWork w;
  w.bg = p->bg;
  // Work items bound the fixed-point deposit sums: <= 2^16 particles (FP32), 2^14 (FP64).
  // FP32 items of 2^15 and one workgroup per item (up to 16384) balance the
  // deposit and gather better than 2^16 and 2048 workgroups looping over
  // items (measured: gather 703 -> 658 us, deposit 394 -> 379 us at 1e8).
  const int64_t item_cap = p->dtype == DKS_F32 ? 32768 : 16384;
  w.bg.item = (int)std::min<int64_t>(item_cap, std::max<int64_t>(8192, maxn / 512));
  w.count_blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (maxn + 8191) / 8192));
  const int64_t items = (maxn + w.bg.item - 1) / w.bg.item + w.bg.K + 1;
  w.item_blocks = (int)std::min<int64_t>(16384, std::max<int64_t>(1, items));
  // kernels never trust more items or particles than the buffers were sized for
  w.bg.max_items = (unsigned)items;
  w.bg.max_np = (unsigned)maxn;
  return w;
}

// Mesh fit (fitted plans), geometry, particle binning and the binned deposit:
// leaves the weights W in R3 and the binned particles in `sorted` (or, soa,
// in the caller's output position arrays soa[0..2]).
template <typename T>
dks_status deposit_stage(const dks_poisson_plan_s* p, int batch, const Slots& sl, const ElemBatch& eb,
                         char* sorted, size_t sorted_stride, size_t inv_off, const PartWork& w,
                         hipStream_t st, void* const* soa = nullptr) {
  int nb = 0;
  double* bbox = reinterpret_cast<double*>(sl.base + p->s_bbox);
  if (p->fitted) DKS_TK("bbox", launch_bbox<T>(eb, batch, bbox, sl.stride / sizeof(double), &nb, st));
  GeoArgs ga = geo_args(p, 1, nb);
  ga.zero_off = p->s_bins;                  // the per-group tile counts
  ga.zero_len = kXcd * (p->bg.K + 1);
  // The order-independent deposit sums into integer node totals in R2
  // (free until the forward y pass) and forms W from them afterwards.
  const size_t nmesh = (size_t)p->n[0] * p->n[1] * p->n[2];
  char* iacc = p->deterministic ? sl.base + p->s_r2 : nullptr;
  const size_t iacc_bytes = nmesh * (sizeof(T) == 4 ? 8 : 16);
  DKS_TK("geometry", launch_geometry_zero(bbox, sl.stride / sizeof(double), sl.geo(), sl.stride, ga, eb, batch,
                                          iacc ? iacc : sl.base + p->s_r3, sl.stride, iacc ? iacc_bytes : p->bytes_W,
                                          st));
  DKS_TK("bin_count", launch_bin_count<T>(eb, batch, sl.geo(), sl.stride, sl.base, p->s_bins, p->md, w.bg,
                                          w.count_blocks, st));
  DKS_TK("bin_scan", launch_bin_scan(sl.geo(), sl.stride, sl.base, p->s_bins, w.bg, eb, batch, st));
  DKS_TK("bin_scatter", launch_bin_scatter<T>(eb, batch, sl.geo(), sl.stride, sl.base, p->s_bins, sorted,
                                              sorted_stride, inv_off, p->md, w.bg, w.count_blocks, soa, st));
  DKS_TK("deposit", launch_deposit_binned<T>(sl.geo(), sl.stride, sl.base, p->s_bins, sorted, sorted_stride,
                                             sl.base + p->s_r3, sl.stride / sizeof(T), p->md, w.bg, w.item_blocks,
                                             batch, soa, iacc, sl.stride / sizeof(unsigned long long), st));
  if (iacc)
    DKS_TK("fixed_to_weights", launch_fixed_to_weights<T>(iacc, sl.stride / sizeof(unsigned long long),
                                                          sl.base + p->s_r3, sl.stride / sizeof(T), nmesh, batch,
                                                          st));
  return DKS_OK;
}

// sorted_out: NULL, or the caller's output arrays (x, y, z, Ex, Ey, Ez,
// new_index or NULL) of a single solve, which then receive the positions
// (written by the scatter, and read back as the binned records) and the
// field in the binned (tile) order instead of the field in the input order,
// and the scatter's inverse permutation.
template <typename T>
dks_status solve_particles_t(const dks_poisson_plan_s* p, int batch, const Slots& sl, const ElemBatch& eb,
                             char* sorted, size_t sorted_stride, hipStream_t st, void* const* sorted_out = nullptr) {
  const PartWork w = part_work(p, eb.max_np);
  const size_t inv_off = inv_offset(p, eb.max_np);
  dks_status r = deposit_stage<T>(p, batch, sl, eb, sorted, sorted_stride, inv_off, w, st, sorted_out);
  if (r != DKS_OK) return r;
  r = convolve<T>(p, sl.base + p->s_r3, sl.stride / sizeof(T), batch, sl, eb, st);
  if (r != DKS_OK) return r;
  DKS_TK("gather", launch_gather_binned<T>(sl.geo(), sl.stride, sl.base, p->s_bins, sorted, sorted_stride,
                                           sl.base + p->s_r3, sl.stride / sizeof(T), p->md, w.bg, w.item_blocks,
                                           batch, sorted_out, st));
  if (!sorted_out) DKS_TK("unsort", launch_unsort<T>(eb, batch, sorted, sorted_stride, inv_off, st));
  return DKS_OK;
}

// No particles (mesh-only geometry).
ElemBatch no_elements() {
  ElemBatch eb;
  std::memset(&eb, 0, sizeof(eb));
  return eb;
}

template <typename T>
dks_status prepare_t(dks_poisson_plan_s* p, hipStream_t st) {
  const size_t c = p->csize;
  (void)c;
  const FFTPlanHost* plans[4] = {&p->px, &p->py, &p->pz, &p->pzi};
  const size_t offs[4] = {p->tw_px, p->tw_py, p->tw_pz, p->tw_pzi};
  for (int i = 0; i < 4; ++i) {
    const FFTPlan& f = plans[i]->dev;
    for (int q = 1; q < f.npass; ++q)
      DKS_CK(launch_twiddle_pass<T>(p->ws + offs[i] + (size_t)f.tw_off[q] * p->csize, f.Ns[q], f.R[q], st));
  }
  DKS_CK(launch_twiddle_line<T>(p->ws + p->tw_post, 2 * p->n[0], p->n[0] + 1, st));
  FFTPlan four[4];
  for (int i = 0; i < 4; ++i) four[i] = planref(p, i).host;
  DKS_CK(launch_store_plans(four, reinterpret_cast<FFTPlan*>(p->ws + p->off_plans), st));
  char* slot = p->ws + p->off_slot;
  double* g1 = reinterpret_cast<double*>(slot + p->s_r1);
  double* g2 = reinterpret_cast<double*>(slot + p->s_r2);
  double* cosm = reinterpret_cast<double*>(slot + p->s_r3);
  double* cos_axis[3];
  cos_axis[0] = cosm;
  cos_axis[1] = cos_axis[0] + (size_t)(p->n[0] + 1) * (p->n[0] + 1);
  cos_axis[2] = cos_axis[1] + (size_t)(p->n[1] + 1) * (p->n[1] + 1);
  const double hg[3] = {p->fitted ? 1.0 : p->h[0], p->fitted ? 1.0 : p->h[1], p->fitted ? 1.0 : p->h[2]};
  const GLBands gl = make_bands();
  DKS_CK(launch_igf_octant(g1, p->n, hg, gl, p->green == DKS_GREEN_POINT ? 1 : 0, st));
  for (int d = 0; d < 3; ++d) DKS_CK(launch_cos_matrix(cos_axis[d], p->n[d], st));
  DKS_CK(launch_apply_axis(g1, g2, cos_axis[0], p->n, 0, st));
  DKS_CK(launch_apply_axis(g2, g1, cos_axis[1], p->n, 1, st));
  DKS_CK(launch_apply_axis(g1, g2, cos_axis[2], p->n, 2, st));
  const double inv_ntot = 1.0 / ((double)(2 * p->n[0]) * (double)(2 * p->n[1]) * (double)(2 * p->n[2]));
  DKS_CK(launch_green_pack<T>(g2, p->ws + p->off_green, p->n, p->md.cs, p->pz.dev.W, inv_ntot, st));
  if (!p->fitted) {
    const GeoArgs ga = geo_args(p, 0, 0);
    DKS_CK(launch_geometry(nullptr, 0, reinterpret_cast<Geometry*>(slot), 0, ga, no_elements(), 1, st));
  }
  return DKS_OK;
}

bool ws_ready(const dks_poisson_plan_s* p) { return p->ws != nullptr && p->ws_bytes >= p->ws_total; }

// One element described by value (single solves).
ElemBatch single(const void* x, const void* y, const void* z, void* ex, void* ey, void* ez, void* phi,
                 int64_t* n_outside, int64_t np, double q, bool need_e) {
  ElemBatch eb;
  std::memset(&eb, 0, sizeof(eb));
  eb.local.x = x;
  eb.local.y = y;
  eb.local.z = z;
  eb.local.Ex = ex;
  eb.local.Ey = ey;
  eb.local.Ez = ez;
  eb.local.phi = phi;
  eb.local.n_outside = n_outside;
  eb.local.np = np;
  eb.local.q = q;
  eb.max_np = np;
  eb.need_e = need_e ? 1 : 0;
  return eb;
}

// rho (device) -> phi and/or E_mesh (device) on an explicit-h plan.
dks_status solve_rho_dev(dks_poisson_plan_s* p, const void* rho, void* phi, void* E_mesh, hipStream_t st) {
  Slots sl{p->ws + p->off_slot, p->slot_bytes};
  const GeoArgs ga = geo_args(p, 0, 0);
  if (launch_geometry(nullptr, 0, sl.geo(), sl.stride, ga, no_elements(), 1, st) != hipSuccess) return DKS_EHIP;
  const ElemBatch out = single(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, phi, nullptr, 0, 0.0, false);
  dks_status r;
  if (p->dtype == DKS_F32) {
    r = convolve<float>(p, rho, 0, 1, sl, out, st);
    if (r == DKS_OK && E_mesh) {
      Timed tm("gradient", st);
      r = hip_status(launch_gradient<float>(sl.base + p->s_r3, E_mesh, sl.geo(), p->md, st));
      tm.done();
    }
  } else {
    r = convolve<double>(p, rho, 0, 1, sl, out, st);
    if (r == DKS_OK && E_mesh) {
      Timed tm("gradient", st);
      r = hip_status(launch_gradient<double>(sl.base + p->s_r3, E_mesh, sl.geo(), p->md, st));
      tm.done();
    }
  }
  if (r == DKS_OK) p->has_geometry = true;
  return r;
}

// Host staging: per slot rho, phi, E (3 components), each array 256-aligned.
size_t mesh_unit(const dks_poisson_plan_s* p) {
  return align256((size_t)p->n[0] * p->n[1] * p->n[2] * p->rsize);
}
size_t host_stage_bytes(const dks_poisson_plan_s* p) { return 2 * 5 * mesh_unit(p); }

// Wait for every issued host-resident solve, then release streams and events.
void host_pipe_release(HostPipe& hp) {
  if (hp.up) (void)hipStreamSynchronize(hp.up);
  if (hp.down) (void)hipStreamSynchronize(hp.down);
  for (int b = 0; b < 2; ++b) {
    if (hp.computed[b]) (void)hipEventDestroy(hp.computed[b]);
    if (hp.uploaded[b]) (void)hipEventDestroy(hp.uploaded[b]);
    hp.computed[b] = hp.uploaded[b] = nullptr;
  }
  for (int i = 0; i < kHostRing; ++i) {
    if (hp.landed[i]) (void)hipEventDestroy(hp.landed[i]);
    hp.landed[i] = nullptr;
  }
  if (hp.up) (void)hipStreamDestroy(hp.up);
  if (hp.down) (void)hipStreamDestroy(hp.down);
  hp.up = hp.down = nullptr;
}

// Streams and events of the host pipeline, created once on the current device
// (all or nothing: a failure releases what was made).
dks_status host_pipe_init(HostPipe& hp) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DKS_EHIP;
  if (hp.device >= 0) return hp.device == dev ? DKS_OK : DKS_EINVAL;
  bool ok = hipStreamCreateWithFlags(&hp.up, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&hp.down, hipStreamNonBlocking) == hipSuccess;
  for (int b = 0; ok && b < 2; ++b)
    ok = hipEventCreateWithFlags(&hp.computed[b], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&hp.uploaded[b], hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < kHostRing; ++i)
    ok = hipEventCreateWithFlags(&hp.landed[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    host_pipe_release(hp);
    return DKS_EHIP;
  }
  hp.device = dev;
  return DKS_OK;
}

// The event that is complete once `ticket` has landed: its own while it is
// still in the ring, else the oldest ticket in the ring (in-order landing).
hipEvent_t landed_event(const HostPipe& hp, uint64_t ticket) {
  const uint64_t oldest = hp.issued > (uint64_t)kHostRing ? hp.issued - kHostRing : 0;
  return hp.landed[std::max(ticket, oldest) % kHostRing];
}

}  // namespace

// Binned-particle scratch of the allocation-free particle solve: a file-scope
// device array (each GPU the library runs on holds its own copy until the
// process ends).  Host code never uses the array's name as an address: its
// device address is looked up once per device with hipGetSymbolAddress.
constexpr size_t kNoallocScratchBytes = (size_t)DKS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up on the first call on it.
static dks_status noalloc_scratch(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return DKS_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return DKS_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DKS_EHIP;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return DKS_OK;
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* dks_status_string(dks_status s) {
  switch (s) {
    case DKS_OK: return "success";
    case DKS_EINVAL: return "invalid argument";
    case DKS_EUNSUPPORTED: return "unsupported mesh size (each 2n must be 2^a 3^b and <= 4096)";
    case DKS_ENOMEM: return "host allocation failed";
    case DKS_EHIP: return "HIP runtime error";
    case DKS_EWORKSPACE: return "workspace missing, too small or misaligned";
    case DKS_ESTATE: return "call out of order for this plan";
  }
  return "unknown status";
}

dks_status dks_poisson_plan(int nx, int ny, int nz, double hx, double hy, double hz, dks_dtype dtype,
                            dks_poisson_plan_t* out) {
  if (!out) return DKS_EINVAL;
  *out = nullptr;
  if (dtype != DKS_F32 && dtype != DKS_F64) return DKS_EINVAL;
  const bool fitted = (hx == 0.0 && hy == 0.0 && hz == 0.0);
  const double hs[3] = {hx, hy, hz};
  if (!fitted)
    for (double h : hs)
      if (!(h > 0.0) || !std::isfinite(h)) return DKS_EINVAL;
  const int ns[3] = {nx, ny, nz};
  for (int n : ns) {
    if (n < (fitted ? 4 : 2)) return DKS_EINVAL;
    if (n > kMaxLength / 2 || !factor23(2 * n)) return DKS_EUNSUPPORTED;
  }
  dks_poisson_plan_s* p = new (std::nothrow) dks_poisson_plan_s;
  if (!p) return DKS_ENOMEM;
  std::memset(p, 0, sizeof(*p));
  for (int d = 0; d < 3; ++d) {
    p->n[d] = ns[d];
    p->h[d] = fitted ? 1.0 : hs[d];
    p->origin[d] = fitted ? 0.0 : -0.5 * (ns[d] - 1) * hs[d];
  }
  p->fitted = fitted;
  p->dtype = dtype;
  p->hp.device = -1;
  p->rsize = dtype == DKS_F32 ? sizeof(float) : sizeof(double);
  p->csize = 2 * p->rsize;
  try {
    layout(p);
  } catch (...) {
    delete p;
    return DKS_ENOMEM;
  }
  if (check_plans(p) != kPlanOk) {
    delete p;
    return DKS_EUNSUPPORTED;
  }
  *out = p;
  return DKS_OK;
}

dks_status dks_poisson_set_origin(dks_poisson_plan_t p, double x0, double y0, double z0) {
  if (!p) return DKS_EINVAL;
  if (p->fitted) return DKS_ESTATE;
  if (!std::isfinite(x0) || !std::isfinite(y0) || !std::isfinite(z0)) return DKS_EINVAL;
  p->origin[0] = x0;
  p->origin[1] = y0;
  p->origin[2] = z0;
  return DKS_OK;
}

dks_status dks_poisson_set_scheme(dks_poisson_plan_t p, dks_green green, dks_assign assign) {
  if (!p) return DKS_EINVAL;
  if (green != DKS_GREEN_INTEGRATED && green != DKS_GREEN_POINT) return DKS_EINVAL;
  if (assign != DKS_ASSIGN_CIC && assign != DKS_ASSIGN_NGP && assign != DKS_ASSIGN_TSC) return DKS_EINVAL;
  if ((int)green != p->green) {
    p->green = (int)green;
    p->prepared = false;           // the spectrum must be rebuilt
  }
  p->bg.scheme = assign == DKS_ASSIGN_NGP ? kSchemeNGP : assign == DKS_ASSIGN_TSC ? kSchemeTSC : kSchemeCIC;
  return DKS_OK;
}

dks_status dks_poisson_set_deterministic(dks_poisson_plan_t p, int on) {
  if (!p || (on != 0 && on != 1)) return DKS_EINVAL;
  p->deterministic = on == 1;
  return DKS_OK;
}

dks_status dks_poisson_workspace_bytes(dks_poisson_plan_t p, size_t* bytes) {
  if (!p || !bytes) return DKS_EINVAL;
  *bytes = p->ws_total;
  return DKS_OK;
}

dks_status dks_poisson_particle_scratch_bytes(dks_poisson_plan_t p, int64_t np, size_t* bytes) {
  if (!p || !bytes || np < 0 || np > kMaxParticles) return DKS_EINVAL;
  *bytes = particle_bytes(p, np);
  return DKS_OK;
}

dks_status dks_poisson_set_particle_scratch(dks_poisson_plan_t p, void* buf, size_t bytes) {
  if (!p) return DKS_EINVAL;
  if (bytes > 0 && (!buf || (reinterpret_cast<uintptr_t>(buf) & 255u))) return DKS_EWORKSPACE;
  p->pscratch = static_cast<char*>(buf);
  p->pscratch_bytes = buf ? bytes : 0;
  return DKS_OK;
}

dks_status dks_poisson_batch_scratch_bytes(dks_poisson_plan_t p, int batch, int64_t max_np, size_t* bytes) {
  if (!p || !bytes || batch < 1 || batch > kMaxBatch || max_np < 0 || max_np > kMaxParticles)
    return DKS_EINVAL;
  *bytes = (size_t)batch * (p->slot_bytes + particle_bytes(p, max_np));
  return DKS_OK;
}

dks_status dks_poisson_set_workspace(dks_poisson_plan_t p, void* ws, size_t bytes) {
  if (!p) return DKS_EINVAL;
  if (!ws || bytes < p->ws_total || (reinterpret_cast<uintptr_t>(ws) & 255u)) return DKS_EWORKSPACE;
  p->ws = static_cast<char*>(ws);
  p->ws_bytes = bytes;
  p->prepared = false;
  p->has_geometry = false;
  return DKS_OK;
}

dks_status dks_poisson_prepare(dks_poisson_plan_t p, dks_stream_t stream) {
  if (!p) return DKS_EINVAL;
  if (!ws_ready(p)) return DKS_EWORKSPACE;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const dks_status r = p->dtype == DKS_F32 ? prepare_t<float>(p, st) : prepare_t<double>(p, st);
  if (r == DKS_OK) {
    p->prepared = true;
    p->has_geometry = !p->fitted;
  }
  return r;
}

dks_status dks_poisson_solve_rho(dks_poisson_plan_t p, const void* rho, void* phi, void* E_mesh,
                                 dks_stream_t stream) {
  if (!p || !rho || (!phi && !E_mesh)) return DKS_EINVAL;
  if (p->fitted) return DKS_ESTATE;
  if (!ws_ready(p)) return DKS_EWORKSPACE;
  if (!p->prepared) return DKS_ESTATE;
  return solve_rho_dev(p, rho, phi, E_mesh, static_cast<hipStream_t>(stream));
}

dks_status dks_poisson_host_staging_bytes(dks_poisson_plan_t p, size_t* bytes) {
  if (!p || !bytes) return DKS_EINVAL;
  *bytes = host_stage_bytes(p);
  return DKS_OK;
}

dks_status dks_poisson_set_host_staging(dks_poisson_plan_t p, void* staging, size_t bytes) {
  if (!p || !staging) return DKS_EINVAL;
  if (bytes < host_stage_bytes(p) || (reinterpret_cast<uintptr_t>(staging) & 255) != 0) return DKS_EWORKSPACE;
  HostPipe& hp = p->hp;
  if (hp.device >= 0 && (hipStreamSynchronize(hp.up) != hipSuccess || hipStreamSynchronize(hp.down) != hipSuccess))
    return DKS_EHIP;
  hp.stage = static_cast<char*>(staging);
  hp.stage_bytes = bytes;
  return DKS_OK;
}

dks_status dks_poisson_solve_rho_host(dks_poisson_plan_t p, const void* rho_host, void* phi_host, void* E_host,
                                      dks_stream_t stream, uint64_t* ticket) {
  if (!p || !rho_host || (!phi_host && !E_host) || !ticket) return DKS_EINVAL;
  if (p->fitted || !p->prepared) return DKS_ESTATE;
  if (!ws_ready(p) || !p->hp.stage) return DKS_EWORKSPACE;
  HostPipe& hp = p->hp;
  const dks_status ri = host_pipe_init(hp);
  if (ri != DKS_OK) return ri;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const uint64_t k = hp.issued;
  const int b = (int)(k & 1);
  const size_t u = mesh_unit(p);
  const size_t mesh = (size_t)p->n[0] * p->n[1] * p->n[2] * p->rsize;
  char* rho_d = hp.stage + (size_t)b * 5 * u;
  char* phi_d = rho_d + u;
  char* E_d = rho_d + 2 * u;
  // upload into slot b once solve k-2 has finished reading it
  if (k >= 2 && hipStreamWaitEvent(hp.up, hp.computed[b], 0) != hipSuccess) return DKS_EHIP;
  if (hipMemcpyAsync(rho_d, rho_host, mesh, hipMemcpyHostToDevice, hp.up) != hipSuccess) return DKS_EHIP;
  if (hipEventRecord(hp.uploaded[b], hp.up) != hipSuccess) return DKS_EHIP;
  // compute once the input is there and solve k-2's outputs have left slot b
  if (hipStreamWaitEvent(st, hp.uploaded[b], 0) != hipSuccess) return DKS_EHIP;
  if (k >= 2 && hipStreamWaitEvent(st, hp.landed[(k - 2) % kHostRing], 0) != hipSuccess) return DKS_EHIP;
  const dks_status rc = solve_rho_dev(p, rho_d, phi_host ? phi_d : nullptr, E_host ? E_d : nullptr, st);
  if (rc != DKS_OK) return rc;
  if (hipEventRecord(hp.computed[b], st) != hipSuccess) return DKS_EHIP;
  // download
  if (hipStreamWaitEvent(hp.down, hp.computed[b], 0) != hipSuccess) return DKS_EHIP;
  if (phi_host && hipMemcpyAsync(phi_host, phi_d, mesh, hipMemcpyDeviceToHost, hp.down) != hipSuccess)
    return DKS_EHIP;
  if (E_host && hipMemcpyAsync(E_host, E_d, 3 * mesh, hipMemcpyDeviceToHost, hp.down) != hipSuccess)
    return DKS_EHIP;
  if (hipEventRecord(hp.landed[k % kHostRing], hp.down) != hipSuccess) return DKS_EHIP;
  hp.issued = k + 1;
  *ticket = k;
  return DKS_OK;
}

dks_status dks_poisson_host_query(dks_poisson_plan_t p, uint64_t ticket, int* done) {
  if (!p || !done || ticket >= p->hp.issued) return DKS_EINVAL;
  const hipError_t e = hipEventQuery(landed_event(p->hp, ticket));
  if (e == hipSuccess) {
    *done = 1;
    return DKS_OK;
  }
  if (e == hipErrorNotReady) {
    *done = 0;
    return DKS_OK;
  }
  return DKS_EHIP;
}

dks_status dks_poisson_host_wait(dks_poisson_plan_t p, uint64_t ticket) {
  if (!p || ticket >= p->hp.issued) return DKS_EINVAL;
  return hipEventSynchronize(landed_event(p->hp, ticket)) == hipSuccess ? DKS_OK : DKS_EHIP;
}

dks_status dks_poisson_solve_particles(dks_poisson_plan_t p, const void* x, const void* y, const void* z,
                                       int64_t np, double q, void* Ex, void* Ey, void* Ez, void* phi,
                                       int64_t* n_outside, dks_stream_t stream) {
  if (!p || np < 0 || np > kMaxParticles || !std::isfinite(q)) return DKS_EINVAL;
  if (np > 0 && (!x || !y || !z || !Ex || !Ey || !Ez)) return DKS_EINVAL;
  if (!ws_ready(p)) return DKS_EWORKSPACE;
  if (particle_bytes(p, np) > p->pscratch_bytes) return DKS_EWORKSPACE;
  if (!p->prepared) return DKS_ESTATE;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  Slots sl{p->ws + p->off_slot, p->slot_bytes};
  const ElemBatch eb = single(x, y, z, Ex, Ey, Ez, phi, n_outside, np, q, true);
  const dks_status r = p->dtype == DKS_F32 ? solve_particles_t<float>(p, 1, sl, eb, p->pscratch, 0, st)
                                           : solve_particles_t<double>(p, 1, sl, eb, p->pscratch, 0, st);
  if (r == DKS_OK) p->has_geometry = true;
  return r;
}

dks_status dks_poisson_solve_particles_noalloc(dks_poisson_plan_t p, const void* x, const void* y, const void* z,
                                               int64_t np, double q, void* Ex, void* Ey, void* Ez, void* phi,
                                               int64_t* n_outside, dks_stream_t stream) {
  if (!p || np < 0 || np > kMaxParticles || !std::isfinite(q)) return DKS_EINVAL;
  if (np > 0 && (!x || !y || !z || !Ex || !Ey || !Ez)) return DKS_EINVAL;
  if (!ws_ready(p)) return DKS_EWORKSPACE;
  if (particle_bytes(p, np) > kNoallocScratchBytes) return DKS_EWORKSPACE;
  if (!p->prepared) return DKS_ESTATE;
  char* buf = nullptr;
  const dks_status rs = noalloc_scratch(&buf);
  if (rs != DKS_OK) return rs;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  Slots sl{p->ws + p->off_slot, p->slot_bytes};
  const ElemBatch eb = single(x, y, z, Ex, Ey, Ez, phi, n_outside, np, q, true);
  const dks_status r = p->dtype == DKS_F32 ? solve_particles_t<float>(p, 1, sl, eb, buf, 0, st)
                                           : solve_particles_t<double>(p, 1, sl, eb, buf, 0, st);
  if (r == DKS_OK) p->has_geometry = true;
  return r;
}

dks_status dks_poisson_solve_particles_sorted(dks_poisson_plan_t p, const void* x, const void* y, const void* z,
                                              int64_t np, double q, void* x_out, void* y_out, void* z_out, void* Ex,
                                              void* Ey, void* Ez, void* phi, uint32_t* new_index,
                                              int64_t* n_outside, dks_stream_t stream) {
  if (!p || np < 0 || np > kMaxParticles || !std::isfinite(q)) return DKS_EINVAL;
  if (np > 0 && (!x || !y || !z || !x_out || !y_out || !z_out || !Ex || !Ey || !Ez)) return DKS_EINVAL;
  if (np > 0) {
    // the outputs are written while the inputs are still being read, and
    // the position outputs are read back as the binned records
    const void* arr[10] = {new_index, x_out, y_out, z_out, Ex, Ey, Ez, x, y, z};
    auto bytes = [&](int i) { return (size_t)np * (i == 0 ? sizeof(uint32_t) : (size_t)p->rsize); };
    for (int i = new_index ? 0 : 1; i < 7; ++i)
      for (int j = i + 1; j < 10; ++j) {
        const char* a = static_cast<const char*>(arr[i]);
        const char* b = static_cast<const char*>(arr[j]);
        if (a < b + bytes(j) && b < a + bytes(i)) return DKS_EINVAL;
      }
  }
  if (!ws_ready(p)) return DKS_EWORKSPACE;
  if (particle_bytes(p, np) > p->pscratch_bytes) return DKS_EWORKSPACE;
  if (!p->prepared) return DKS_ESTATE;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  Slots sl{p->ws + p->off_slot, p->slot_bytes};
  const ElemBatch eb = single(x, y, z, Ex, Ey, Ez, phi, n_outside, np, q, true);
  // the scatter writes the new position of each input index straight into
  // new_index (and no inverse permutation at all when it is NULL)
  void* const outs[7] = {x_out, y_out, z_out, Ex, Ey, Ez, new_index};
  const dks_status r = p->dtype == DKS_F32 ? solve_particles_t<float>(p, 1, sl, eb, p->pscratch, 0, st, outs)
                                           : solve_particles_t<double>(p, 1, sl, eb, p->pscratch, 0, st, outs);
  if (r != DKS_OK) return r;
  p->has_geometry = true;
  return DKS_OK;
}

dks_status dks_poisson_solve_particles_batched(dks_poisson_plan_t p, int batch, const dks_particle_set* sets,
                                               int64_t max_np, void* buf, size_t buf_bytes,
                                               dks_stream_t stream) {
  if (!p || batch < 1 || batch > kMaxBatch || !sets) return DKS_EINVAL;
  if (max_np < 0 || max_np > kMaxParticles) return DKS_EINVAL;
  if (!ws_ready(p)) return DKS_EWORKSPACE;
  if (!p->prepared) return DKS_ESTATE;
  if (!buf || (reinterpret_cast<uintptr_t>(buf) & 255u)) return DKS_EWORKSPACE;
  // Element b owns [b * stride, (b + 1) * stride): its slot, then its binned particles.
  const size_t stride = (buf_bytes / (size_t)batch) & ~(size_t)255;
  if (stride < p->slot_bytes + particle_bytes(p, max_np)) return DKS_EWORKSPACE;
  ElemBatch eb;
  std::memset(&eb, 0, sizeof(eb));
  eb.dev = sets;
  eb.max_np = max_np;
  eb.need_e = 1;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  Slots sl{static_cast<char*>(buf), stride};
  char* sorted = static_cast<char*>(buf) + p->slot_bytes;
  return p->dtype == DKS_F32 ? solve_particles_t<float>(p, batch, sl, eb, sorted, stride, st)
                             : solve_particles_t<double>(p, batch, sl, eb, sorted, stride, st);
}

dks_status dks_poisson_deposit(dks_poisson_plan_t p, const void* x, const void* y, const void* z, int64_t np,
                               double q, void* rho, int64_t* n_outside, dks_stream_t stream) {
  if (!p || !rho || np < 0 || np > kMaxParticles || !std::isfinite(q)) return DKS_EINVAL;
  if (np > 0 && (!x || !y || !z)) return DKS_EINVAL;
  if (!ws_ready(p)) return DKS_EWORKSPACE;
  if (particle_bytes(p, np) > p->pscratch_bytes) return DKS_EWORKSPACE;
  if (!p->prepared) return DKS_ESTATE;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  Slots sl{p->ws + p->off_slot, p->slot_bytes};
  const ElemBatch eb = single(x, y, z, nullptr, nullptr, nullptr, nullptr, n_outside, np, q, false);
  const PartWork w = part_work(p, np);
  const size_t nmesh = (size_t)p->n[0] * p->n[1] * p->n[2];
  dks_status r;
  if (p->dtype == DKS_F32) {
    r = deposit_stage<float>(p, 1, sl, eb, p->pscratch, 0, inv_offset(p, np), w, st);
    if (r == DKS_OK) r = hip_status(launch_weights_to_density<float>(sl.base + p->s_r3, rho, nmesh, sl.geo(), q, st));
  } else {
    r = deposit_stage<double>(p, 1, sl, eb, p->pscratch, 0, inv_offset(p, np), w, st);
    if (r == DKS_OK) r = hip_status(launch_weights_to_density<double>(sl.base + p->s_r3, rho, nmesh, sl.geo(), q, st));
  }
  if (r == DKS_OK) p->has_geometry = true;
  return r;
}

dks_status dks_poisson_gather(dks_poisson_plan_t p, const void* E_mesh, const void* x, const void* y,
                              const void* z, int64_t np, void* Ex, void* Ey, void* Ez, dks_stream_t stream) {
  if (!p || !E_mesh || np < 0) return DKS_EINVAL;
  if (np > 0 && (!x || !y || !z || !Ex || !Ey || !Ez)) return DKS_EINVAL;
  if (!ws_ready(p)) return DKS_EWORKSPACE;
  if (!p->prepared) return DKS_ESTATE;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  Slots sl{p->ws + p->off_slot, p->slot_bytes};
  if (!p->fitted) {
    const GeoArgs ga = geo_args(p, 0, 0);
    if (launch_geometry(nullptr, 0, sl.geo(), sl.stride, ga, no_elements(), 1, st) != hipSuccess) return DKS_EHIP;
  } else if (!p->has_geometry) {
    return DKS_ESTATE;
  }
  if (p->dtype == DKS_F32)
    return hip_status(launch_gather<float>(E_mesh, x, y, z, Ex, Ey, Ez, np, sl.geo(), p->md, p->bg.scheme, st));
  return hip_status(launch_gather<double>(E_mesh, x, y, z, Ex, Ey, Ez, np, sl.geo(), p->md, p->bg.scheme, st));
}

dks_status dks_poisson_geometry(dks_poisson_plan_t p, dks_stream_t stream, double* h, double* origin) {
  if (!p || !h || !origin) return DKS_EINVAL;
  if (!ws_ready(p)) return DKS_EWORKSPACE;
  if (!p->has_geometry) return DKS_ESTATE;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  Geometry g;
  if (hipMemcpyAsync(&g, p->ws + p->off_slot, sizeof(Geometry), hipMemcpyDeviceToHost, st) != hipSuccess)
    return DKS_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return DKS_EHIP;
  for (int d = 0; d < 3; ++d) {
    h[d] = g.h[d];
    origin[d] = g.origin[d];
  }
  return DKS_OK;
}

dks_status dks_timing_enable(int enable) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> lock(t.mu);
  for (auto& r : t.recs) (void)hipEventSynchronize(r.b);
  t.release_all();
  t.on = enable != 0;
  return DKS_OK;
}

dks_status dks_timing_read(dks_kernel_time* out, int capacity, int* count) {
  if (!count || capacity < 0 || (capacity > 0 && !out)) return DKS_EINVAL;
  TimingState& t = timing();
  std::lock_guard<std::mutex> lock(t.mu);
  std::map<std::string, dks_kernel_time> agg;
  std::vector<std::string> order;
  for (auto& r : t.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return DKS_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return DKS_EHIP;
    auto it = agg.find(r.name);
    if (it == agg.end()) {
      dks_kernel_time k;
      std::memset(&k, 0, sizeof(k));
      std::strncpy(k.name, r.name, sizeof(k.name) - 1);
      k.min_ms = ms;
      k.max_ms = ms;
      it = agg.emplace(r.name, k).first;
      order.push_back(r.name);
    }
    it->second.launches += 1;
    it->second.total_ms += ms;
    it->second.min_ms = std::min(it->second.min_ms, (double)ms);
    it->second.max_ms = std::max(it->second.max_ms, (double)ms);
  }
  *count = (int)order.size();
  if ((int)order.size() > capacity) return DKS_EINVAL;
  for (size_t i = 0; i < order.size(); ++i) out[i] = agg[order[i]];
  t.release_all();
  return DKS_OK;
}

dks_status dks_poisson_destroy(dks_poisson_plan_t p) {
  if (!p) return DKS_EINVAL;
  host_pipe_release(p->hp);
  delete p;
  return DKS_OK;
}

}  // extern "C"
