// Spatially binned cloud-in-cell deposit and gather.
//
// A compact bunch puts hundreds of particles in each central cell, so a
// deposit that adds every particle's eight weights straight into the mesh
// with device-wide atomics serialises on the hot nodes, and a gather over
// unsorted particles reads the mesh at random.  Both steps here work on the
// particles grouped by the 16^3-cell tile that holds their CIC cell:
//
//   count    per-tile histogram (LDS-privatised, flushed with one atomic per
//            touched tile per workgroup)
//   scan     tile offsets, reservation cursors and the work-item list
//            (a work item is up to kItem particles of one tile)
//   scatter  one workgroup per chunk of 8192 (FP32) / 4096 (FP64) consecutive
//            particles: ranks within tiles from an LDS histogram, one device
//            atomic per touched tile to reserve the chunk's range, then the
//            particles are written there as packed (x, y, z) records and the
//            inverse permutation (original index -> binned slot) is written
//            in original order
//   deposit  per work item: accumulate the weights of the tile's particles in
//            an LDS copy of its 17^3 nodes with integer LDS atomics on a fixed-
//            point scale (exact and order independent; floating-point LDS
//            atomics run an order of magnitude slower), then merge the copy
//            into the mesh with one device atomic per non-zero node
//   gather   per work item: stage phi of the tile plus a two-node apron
//            (19^3 values) in LDS, form the central-difference field at the
//            eight nodes of each particle and interpolate it with the
//            deposit's weights; the field overwrites the particle's binned
//            record in place
//   unsort   per scatter chunk, read each field through the inverse
//            permutation and write the three field arrays contiguously; a
//            chunk's records lie in one short segment per touched tile, so
//            its scattered 16-byte reads share cache lines (scattered 4-byte
//            writes to the original indices would cost far more)
//
// Particles outside the mesh fall in an extra tile K: they deposit nothing,
// get E = 0 and their count is the out-of-mesh count.  The cell decision is
// made from the same (x - x0) * (1/h) in the dtype as everywhere else, so the
// tile a particle is filed under always contains its whole stencil.

#include <math.h>

#include <algorithm>
#include <type_traits>

#include "dks_internal.h"

namespace dks {

constexpr int kTile = 16;          // cells per tile edge
// Per tile edge: deposit accumulator nodes (the tile's stencil reach) and
// staged phi values of the gather (one more node on each side for the
// central differences).  CIC: 17 and 19; NGP: 16 and 18; TSC: 18 and 20.
template <int SCH> constexpr int acc_edge() { return kTile + Scheme<SCH>::width - 1; }
template <int SCH> constexpr int apron_edge() { return acc_edge<SCH>() + 2; }

// Lanes per deposit / gather workgroup: the LDS tile bounds the workgroups
// per CU, so wider workgroups keep more record loads in flight.
constexpr int kDepositThreads = 1024;
constexpr int kGatherThreads = 512;

// Binned records each lane loads before using any.
constexpr int kUnrollDeposit = 4;
constexpr int kUnrollGather = 2;

// A binned particle record: its position, overwritten by the field at it.
template <typename T> struct Rec {
  T x, y, z;
};

// Caller arrays of the tile-ordered step (one element): x, y, z receive the
// positions in binned order and serve as the binned records themselves;
// ex, ey, ez receive the field in that order; inv (or NULL: not written)
// receives the new position of each input index.
template <typename T> struct SortedOut {
  T* x;
  T* y;
  T* z;
  T* ex;
  T* ey;
  T* ez;
  unsigned* inv;
};

// The binned records of one element: (x, y, z) records in the particle
// scratch, or (SOA) the three position arrays of a SortedOut.
template <typename T, bool SOA> struct Recs;
template <typename T> struct Recs<T, false> {
  Rec<T>* p;
  __device__ __forceinline__ Rec<T> ld(size_t i) const { return p[i]; }
  __device__ __forceinline__ void st(size_t i, Rec<T> r) const { p[i] = r; }
};
template <typename T> struct Recs<T, true> {
  T* x;
  T* y;
  T* z;
  __device__ __forceinline__ Rec<T> ld(size_t i) const { return Rec<T>{x[i], y[i], z[i]}; }
  __device__ __forceinline__ void st(size_t i, Rec<T> r) const {
    x[i] = r.x;
    y[i] = r.y;
    z[i] = r.z;
  }
};
template <typename T, bool SOA>
__device__ __forceinline__ Recs<T, SOA> recs_of(char* sorted_base, size_t sorted_stride, int b,
                                                const SortedOut<T>& so) {
  if constexpr (SOA) {
    return Recs<T, true>{so.x, so.y, so.z};
  } else {
    return Recs<T, false>{reinterpret_cast<Rec<T>*>(sorted_base + (size_t)b * sorted_stride)};
  }
}

// Fixed-point scale of the deposit accumulators: a weight is at most 1 and a
// work item holds at most 2^16 (FP32) or 2^14 (FP64) particles, so a node sum
// stays below 2^47 resp. 2^63 in 64 bits; the scale keeps 2^-31 resp. 2^-49
// resolution, finer than the dtype's rounding of the weight products.  The
// scale is a power of two, folded exactly into one factor of each product;
// to() takes the scaled weight (an FP32 one fits 32 bits: one rounding
// conversion instead of a 64-bit one).
template <typename T> struct Fixed;
template <> struct Fixed<float> {
  static constexpr float scale = 2147483648.0f;   // 2^31
  static __device__ __forceinline__ unsigned long long to(float ws) { return (unsigned long long)__float2uint_rn(ws); }
  static __device__ __forceinline__ float from(unsigned long long v) { return (float)v * 4.656612873077393e-10f; }
};
template <> struct Fixed<double> {
  static constexpr double scale = 562949953421312.0;   // 2^49
  static __device__ __forceinline__ unsigned long long to(double ws) { return __double2ull_rn(ws); }
  static __device__ __forceinline__ double from(unsigned long long v) { return (double)v * 1.7763568394002505e-15; }
};

__device__ __forceinline__ float cc(float x, float x0, float ih) { return __fmul_rn(__fsub_rn(x, x0), ih); }
__device__ __forceinline__ double cc(double x, double x0, double ih) { return __dmul_rn(__dsub_rn(x, x0), ih); }

__device__ __forceinline__ const Geometry* geo_of(const Geometry* base, size_t stride, int b) {
  return reinterpret_cast<const Geometry*>(reinterpret_cast<const char*>(base) + (size_t)b * stride);
}

__device__ __forceinline__ BinState bin_state(char* slot_base, size_t stride, size_t off, int b, int K) {
  BinState s;
  const int L = K + 1;
  unsigned* p = reinterpret_cast<unsigned*>(slot_base + (size_t)b * stride + off);
  s.xcount = p;
  s.count = p + kXcd * L;
  s.offset = s.count + L;
  s.xcursor = s.offset + L + 1;
  s.item_off = s.xcursor + kXcd * L;
  s.misc = s.item_off + L + 1;
  return s;
}

// Cell decision of one particle: its tile (K if outside), the first node of
// its stencil and the per-axis weights of the assignment scheme.  The tile is
// that of the node axis_stencil files the particle under.
template <typename T, int SCH>
struct Cell {
  int key;
  int bx, by, bz;
  T wx[Scheme<SCH>::width], wy[Scheme<SCH>::width], wz[Scheme<SCH>::width];
};

template <typename T, int SCH>
__device__ __forceinline__ Cell<T, SCH> locate(T x, T y, T z, const Geometry* g, const MeshDims& m,
                                               const BinGeom& bg) {
  Cell<T, SCH> c;
  const T sx = cc(x, Geo<T>::origin(g, 0), Geo<T>::inv_h(g, 0));
  const T sy = cc(y, Geo<T>::origin(g, 1), Geo<T>::inv_h(g, 1));
  const T sz = cc(z, Geo<T>::origin(g, 2), Geo<T>::inv_h(g, 2));
  int kx, ky, kz;
  // every axis is evaluated (its node and weights are set either way)
  const bool inx = axis_stencil<T, SCH>(sx, m.nx, kx, c.wx);
  const bool iny = axis_stencil<T, SCH>(sy, m.ny, ky, c.wy);
  const bool inz = axis_stencil<T, SCH>(sz, m.nz, kz, c.wz);
  const bool in = inx && iny && inz;
  if (in) {
    // node indices are >= 0 here: unsigned division by the tile edge is a shift
    c.key = (int)((((unsigned)kz / kTile) * bg.ty + ((unsigned)ky / kTile)) * bg.tx + ((unsigned)kx / kTile));
    c.bx = kx + Scheme<SCH>::lo;
    c.by = ky + Scheme<SCH>::lo;
    c.bz = kz + Scheme<SCH>::lo;
  } else {
    c.key = bg.K;
    c.bx = c.by = c.bz = 0;
  }
  return c;
}

// Runs f with the scheme as a compile-time constant.
template <class F> __device__ __host__ __forceinline__ void with_scheme(int scheme, F&& f) {
  if (scheme == kSchemeNGP) f(std::integral_constant<int, kSchemeNGP>{});
  else if (scheme == kSchemeTSC) f(std::integral_constant<int, kSchemeTSC>{});
  else f(std::integral_constant<int, kSchemeCIC>{});
}

// Scatter chunks: 8192 (FP32) / 4096 (FP64) consecutive particles.  The
// scatter spreads a chunk over kScatterThreads lanes, the unsort (which
// processes the same chunks, for cache locality) over kUnsortThreads lanes
// with more independent loads per lane.
template <typename T> constexpr int64_t scatter_chunk() { return sizeof(T) == 4 ? 8192 : 4096; }
constexpr int kScatterThreads = 1024;
constexpr int kUnsortThreads = 256;
template <typename T, int THREADS> constexpr int chunk_per() { return (int)(scatter_chunk<T>() / THREADS); }

// Counter increments of one particle per lane, with the lanes of a wavefront
// that share one key served by a single atomic: in tile-ordered input most
// wavefronts hold particles of one tile, and 64 atomics on one LDS address
// serialise (the count pass took 338 us instead of 185 us on such input).
// rank_add returns the counter's old value plus the lane's place among the
// active lanes (lane order), or its own atomic's old value when the keys
// differ; the order of equal keys is arbitrary either way.
__device__ __forceinline__ unsigned rank_add(unsigned* ctr, int key) {
  const int k0 = __builtin_amdgcn_readfirstlane(key);
  if (__all(key == k0)) {
    const unsigned long long act = __ballot(1);
    const int leader = __ffsll((long long)act) - 1;
    const int lane = (int)__lane_id();
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(&ctr[k0], (unsigned)__popcll(act));
    base = __shfl(base, leader);
    return base + (unsigned)__popcll(act & ((1ull << lane) - 1ull));
  }
  return atomicAdd(&ctr[key], 1u);
}
__device__ __forceinline__ void count_add(unsigned* ctr, int key) {
  const int k0 = __builtin_amdgcn_readfirstlane(key);
  if (__all(key == k0)) {
    const unsigned long long act = __ballot(1);
    if ((int)__lane_id() == __ffsll((long long)act) - 1) atomicAdd(&ctr[k0], (unsigned)__popcll(act));
  } else {
    atomicAdd(&ctr[key], 1u);
  }
}

// ---------------------------------------------------------------------------
// count: per XCD group and tile.  Workgroup w walks the scatter chunks
// c = w, w + G, ... (G = gridDim.x, a multiple of kXcd), which all fall in
// group (b * nchunk + w) mod kXcd.
// ---------------------------------------------------------------------------
template <typename T, bool LDSHIST, int SCH>
__global__ __launch_bounds__(256) void k_bin_count(ElemBatch eb, const Geometry* geo, size_t stride, char* slot_base,
                                                   size_t bins_off, MeshDims m, BinGeom bg, int nchunk) {
  extern __shared__ unsigned hist[];
  constexpr int64_t CH = scatter_chunk<T>();
  const int b = blockIdx.y;
  const dks_particle_set e = eb.at(b);
  const T* px = (const T*)e.x;
  const T* py = (const T*)e.y;
  const T* pz = (const T*)e.z;
  const int64_t n = eb.n(e);
  const Geometry* g = geo_of(geo, stride, b);
  BinState st = bin_state(slot_base, stride, bins_off, b, bg.K);
  unsigned* xc = st.xcount + (int)(((int64_t)b * nchunk + blockIdx.x) % kXcd) * (bg.K + 1);
  if (LDSHIST) {
    for (int k = threadIdx.x; k <= bg.K; k += blockDim.x) hist[k] = 0;
    __syncthreads();
  }
  for (int64_t c = blockIdx.x; c * CH < n; c += gridDim.x) {
    for_each_particle<T>(px, py, pz, c * CH, min(c * CH + CH, n), [&](T x, T y, T z, int64_t) {
      const int key = locate<T, SCH>(x, y, z, g, m, bg).key;
      if constexpr (LDSHIST) count_add(hist, key);
      else count_add(xc, key);
    });
  }
  if (LDSHIST) {
    __syncthreads();
    for (int k = threadIdx.x; k <= bg.K; k += blockDim.x)
      if (hist[k]) atomicAdd(&xc[k], hist[k]);
  }
}

// ---------------------------------------------------------------------------
// scan: tile totals, offsets (exclusive prefix over tiles), the per-group
// reservation cursors inside each tile's range, and the work items.  One
// block of 1024 threads per batch element.  Also publishes the out-of-mesh
// count.
// ---------------------------------------------------------------------------
// Exclusive prefix sums of (a, b) over the 1024 lanes of the workgroup in
// lane order: inclusive scans within each wavefront by shuffles, then the
// wavefront totals; returns the exclusive sums, totals in *ta, *tb.
__device__ __forceinline__ void scan1024(unsigned a, unsigned b, unsigned* wa, unsigned* wb, unsigned* ea,
                                         unsigned* eb_, unsigned* ta, unsigned* tb) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned x = a, y = b;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned xo = __shfl_up(x, o, 64), yo = __shfl_up(y, o, 64);
    if (lane >= o) {
      x += xo;
      y += yo;
    }
  }
  if (lane == 63) {
    wa[w] = x;
    wb[w] = y;
  }
  __syncthreads();
  unsigned pa = 0, pb = 0, sa = 0, sb = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i < w) {
      pa += wa[i];
      pb += wb[i];
    }
    sa += wa[i];
    sb += wb[i];
  }
  *ea = pa + x - a;
  *eb_ = pb + y - b;
  *ta = sa;
  *tb = sb;
}

// Tile counts of one element: per-XCD-group counts summed, exclusive offsets,
// per-group reservation cursors, and the work-item list.  Each lane owns a
// contiguous run of tiles; when the run is at most kScanRun tiles (up to
// 8192 tiles, e.g. a 320^3 mesh) its counts stay in registers and all its
// loads are issued together.
constexpr int kScanRun = 8;
__global__ __launch_bounds__(1024) void k_bin_scan(const Geometry* geo, size_t stride, char* slot_base,
                                                   size_t bins_off, BinGeom bg, ElemBatch eb) {
  __shared__ unsigned wa[16], wb[16];
  const int b = blockIdx.x;
  BinState st = bin_state(slot_base, stride, bins_off, b, bg.K);
  const int L = bg.K + 1;
  const int per = (L + 1023) / 1024;
  const int lo = min((int)threadIdx.x * per, L), hi = min(lo + per, L);
  unsigned sc = 0, si = 0, oc, oi, tc, ti;
  if (per <= kScanRun) {
    unsigned c[kScanRun];
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
      c[j] = 0;
      if (lo + j < hi) {
#pragma unroll
        for (int x = 0; x < kXcd; ++x) c[j] += st.xcount[x * L + lo + j];
      }
    }
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
      if (lo + j < hi) {
        st.count[lo + j] = c[j];
        sc += c[j];
        si += (c[j] + bg.item - 1) / bg.item;
      }
    }
    scan1024(sc, si, wa, wb, &oc, &oi, &tc, &ti);
#pragma unroll
    for (int j = 0; j < kScanRun; ++j) {
      const int k = lo + j;
      if (k < hi) {
        st.offset[k] = oc;
        unsigned run = oc;
#pragma unroll
        for (int x = 0; x < kXcd; ++x) {
          st.xcursor[x * L + k] = run;
          run += st.xcount[x * L + k];
        }
        st.item_off[k] = oi;
        oc += c[j];
        oi += (c[j] + bg.item - 1) / bg.item;
      }
    }
  } else {
    for (int k = lo; k < hi; ++k) {
      unsigned c = 0;
#pragma unroll
      for (int x = 0; x < kXcd; ++x) c += st.xcount[x * L + k];
      st.count[k] = c;
      sc += c;
      si += (c + bg.item - 1) / bg.item;
    }
    scan1024(sc, si, wa, wb, &oc, &oi, &tc, &ti);
    for (int k = lo; k < hi; ++k) {
      const unsigned c = st.count[k];
      st.offset[k] = oc;
      unsigned run = oc;
#pragma unroll
      for (int x = 0; x < kXcd; ++x) {
        st.xcursor[x * L + k] = run;
        run += st.xcount[x * L + k];
      }
      st.item_off[k] = oi;
      oc += c;
      oi += (c + bg.item - 1) / bg.item;
    }
  }
  if (threadIdx.x == 1023) {
    st.offset[L] = tc;
    st.item_off[L] = ti;
    st.misc[0] = ti;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long outside = st.count[bg.K];
    int64_t* cnt = eb.at(b).n_outside;
    Geometry* gw = const_cast<Geometry*>(geo_of(geo, stride, b));
    gw->n_outside = outside;
    if (cnt) *cnt = (int64_t)outside;
  }
}

// ---------------------------------------------------------------------------
// scatter: one workgroup per chunk of consecutive particles.  The chunk is
// read once into registers; an LDS histogram gives every particle its rank
// within its tile and the chunk's count per tile; one device atomic per
// touched tile reserves the chunk's range there; then the (x, y, z) records
// and the inverse permutation are written.  A chunk therefore occupies one
// short contiguous segment per touched tile, which is what lets the unsort
// pass read a chunk's records back with few cache lines.
//
// STAGE (the histogram and the whole chunk fit in LDS): the records are first
// placed in LDS in the chunk's own tile order (exclusive scan of the chunk's
// tile counts), then lane p stores record p, so each wavefront's stores cover
// contiguous runs of the destination segments instead of 64 unrelated
// addresses.
// ---------------------------------------------------------------------------

// Particle of slot j (of `per`) of this thread in the chunk starting at c0:
// vector layout (each lane owns 16-byte runs) or element layout.
template <typename T, int THREADS>
__device__ __forceinline__ int64_t chunk_index(bool vec, int64_t c0, int j) {
  constexpr int NV = Vec16<T>::n;
  return vec ? c0 + (int64_t)NV * (threadIdx.x + (j / NV) * THREADS) + (j % NV)
             : c0 + threadIdx.x + (int64_t)j * THREADS;
}

// LDS bytes of the staged scatter: tile counts/offsets and bases, then the
// chunk's records and their tile keys.
template <typename T> constexpr size_t scatter_stage_lds(int K) {
  return 2 * (size_t)(K + 1) * sizeof(unsigned) + (size_t)scatter_chunk<T>() * (sizeof(Rec<T>) + sizeof(unsigned short));
}
constexpr size_t kLdsPerWorkgroup = 160 * 1024;   // gfx950
// Tiles per lane in the staged scan: the staged path needs K + 1 <= 8 * 1024.
constexpr int kStageRun = 8;

// The staged scatter of one chunk, once its keys and ranks are in registers
// and lcnt holds its tile counts (all lanes, after the ranking atomics):
// chunk-local offsets and reservations, records and keys into LDS, the
// inverse permutation, then the records in local order.  Each lane owns a
// contiguous run of at most kStageRun tiles: the chunk-local exclusive
// offsets replace the counts in lcnt, and lbase holds (reserved global start
// - local offset), so that a record's destination is its local position plus
// lbase of its tile.  The lane's reservations are all issued before the scan
// and their results used after it.  FULL: a whole chunk in the vector layout
// (no per-particle checks, vector stores of the inverse permutation); lcnt
// is cleared for the next chunk while the records are stored.  mid() runs
// once the reservations have returned (the pipelined kernel issues the next
// chunk's loads there: issued earlier, waiting for the reservations would
// wait for them too).
struct NoMid {
  __device__ void operator()() const {}
};
template <typename T, bool FULL, class RecOut, class Mid = NoMid, int PER = chunk_per<T, kScatterThreads>()>
__device__ __forceinline__ void scatter_stage_chunk(unsigned* lcnt, unsigned* lbase, Rec<T>* srec,
                                                    unsigned short* skey, unsigned* wa, unsigned* wb,
                                                    unsigned* cursor, const BinGeom& bg, const int (&key)[PER],
                                                    const unsigned (&rank)[PER], const T (&xs)[PER],
                                                    const T (&ys)[PER], const T (&zs)[PER], int64_t c0, int64_t n,
                                                    bool vec, const RecOut& out, unsigned* inv, Mid mid = Mid{}) {
  using P4 = Rec<T>;
  constexpr int NV = Vec16<T>::n;
  constexpr int64_t CH = scatter_chunk<T>();
  __syncthreads();
  const int L = bg.K + 1;
  const int per = (L + kScatterThreads - 1) / kScatterThreads;
  const int lo = min((int)threadIdx.x * per, L), hi = min(lo + per, L);
  unsigned cv[kStageRun], rv[kStageRun];
  unsigned sum = 0;
#pragma unroll
  for (int q = 0; q < kStageRun; ++q) {
    cv[q] = lo + q < hi ? lcnt[lo + q] : 0u;
    sum += cv[q];
  }
#pragma unroll
  for (int q = 0; q < kStageRun; ++q) rv[q] = cv[q] ? atomicAdd(&cursor[lo + q], cv[q]) : 0u;
  unsigned off, unused0, unused1, unused2;
  scan1024(sum, 0u, wa, wb, &off, &unused0, &unused1, &unused2);
#pragma unroll
  for (int q = 0; q < kStageRun; ++q) {
    if (lo + q < hi) {
      lcnt[lo + q] = off;
      lbase[lo + q] = rv[q] - off;
      off += cv[q];
    }
  }
  mid();
  __syncthreads();
  // Records and keys into LDS at their local positions; every destination
  // is formed before the inverse permutation is stored (vector stores of a
  // lane's consecutive particles in the vector layout).
  unsigned dv[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    dv[j] = 0u;
    if (FULL || key[j] >= 0) {
      const unsigned lp = lcnt[key[j]] + rank[j];
      srec[lp] = P4{xs[j], ys[j], zs[j]};
      skey[lp] = (unsigned short)key[j];
      dv[j] = lp + lbase[key[j]];
    }
  }
  if (!inv) {
    // no inverse permutation wanted
  } else if (FULL || vec) {
    struct alignas(NV * sizeof(unsigned)) U { unsigned v[NV]; };
#pragma unroll
    for (int q = 0; q < PER / NV; ++q) {
      const int64_t i = chunk_index<T, kScatterThreads>(true, c0, q * NV);
      if (FULL || i + NV <= n) {
        U u;
#pragma unroll
        for (int k = 0; k < NV; ++k) u.v[k] = dv[q * NV + k];
        *reinterpret_cast<U*>(inv + i) = u;
      } else {
#pragma unroll
        for (int k = 0; k < NV; ++k)
          if (i + k < n) inv[i + k] = dv[q * NV + k];
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int64_t i = chunk_index<T, kScatterThreads>(false, c0, j);
      if (i < n) inv[i] = dv[j];
    }
  }
  __syncthreads();
  if (FULL) {
    for (int k = threadIdx.x; k < L; k += kScatterThreads) lcnt[k] = 0;
  }
  // The chunk's valid particles fill local positions 0 .. nv - 1; a lane
  // reads all of its records before storing any.
  const unsigned nv = FULL ? (unsigned)CH : (unsigned)min(CH, n - c0);   // >= 1
  T rx[PER], ry[PER], rz[PER];
  unsigned dd[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    // lanes past the end re-read the last record and store nothing
    const unsigned p = FULL ? threadIdx.x + (unsigned)j * kScatterThreads
                            : min(threadIdx.x + (unsigned)j * kScatterThreads, nv - 1);
    const P4 r = srec[p];
    rx[j] = r.x;
    ry[j] = r.y;
    rz[j] = r.z;
    dd[j] = p + lbase[skey[p]];
  }
  // Keep the reads above the stores: a store's registers cannot be reused
  // before it completes, so interleaving would serialise the stores.
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int j = 0; j < PER; ++j)
    if (FULL || threadIdx.x + (unsigned)j * kScatterThreads < nv) out.st(dd[j], P4{rx[j], ry[j], rz[j]});
}

template <typename T, bool LDSHIST, bool STAGE, int SCH, bool SOA>
__global__ __launch_bounds__(kScatterThreads) void k_bin_scatter(ElemBatch eb, const Geometry* geo, size_t stride,
                                                                 char* slot_base, size_t bins_off,
                                                                 char* sorted_base, size_t sorted_stride,
                                                                 size_t inv_off, MeshDims m, BinGeom bg,
                                                                 int chunk0, int nchunk, SortedOut<T> so) {
  extern __shared__ unsigned lds[];
  __shared__ unsigned wa[16], wb[16];
  constexpr int PER = chunk_per<T, kScatterThreads>();
  constexpr int NV = Vec16<T>::n;
  constexpr int64_t CH = scatter_chunk<T>();
  static_assert(!STAGE || LDSHIST, "staging needs the LDS histogram");
  using P4 = Rec<T>;
  using V = typename Vec16<T>::type;
  const int b = blockIdx.y;
  const dks_particle_set e = eb.at(b);
  const int64_t n = eb.n(e);
  const int chunk = chunk0 + (int)blockIdx.x;
  const int64_t c0 = (int64_t)chunk * CH;
  if (c0 >= n) return;                       // whole workgroup: no barrier is skipped by part of it
  unsigned* lcnt = lds;
  unsigned* lbase = lds + (bg.K + 1);
  // 2 (K + 1) words precede the records: 8-byte aligned for FP64 records
  P4* srec = reinterpret_cast<P4*>(lds + 2 * (bg.K + 1));
  unsigned short* skey = reinterpret_cast<unsigned short*>(srec + CH);
  const T* px = (const T*)e.x;
  const T* py = (const T*)e.y;
  const T* pz = (const T*)e.z;
  // A private copy of the geometry: the LDS atomics between the particles'
  // cell decisions would otherwise make the compiler reload its fields (and
  // wait for them) once per particle.
  const Geometry gcopy = *geo_of(geo, stride, b);
  const Geometry* g = &gcopy;
  BinState st = bin_state(slot_base, stride, bins_off, b, bg.K);
  // the chunk's XCD group, as the count kernel assigned it
  unsigned* cursor = st.xcursor + (int)(((int64_t)b * nchunk + chunk) % kXcd) * (bg.K + 1);
  const Recs<T, SOA> out = recs_of<T, SOA>(sorted_base, sorted_stride, b, so);
  unsigned* inv = SOA ? so.inv : reinterpret_cast<unsigned*>(sorted_base + (size_t)b * sorted_stride + inv_off);
  if (LDSHIST) {
    for (int k = threadIdx.x; k <= bg.K; k += kScatterThreads) lcnt[k] = 0;
  }
  const bool vec = aligned16(px + c0, py + c0, pz + c0);
  T xs[PER], ys[PER], zs[PER];
  if (vec) {
#pragma unroll
    for (int q = 0; q < PER / NV; ++q) {
      const int64_t i = chunk_index<T, kScatterThreads>(true, c0, q * NV);
      if (i + NV <= n) {
        const V a = ld_stream(px + i), bb = ld_stream(py + i), c = ld_stream(pz + i);
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          xs[q * NV + k] = a[k];
          ys[q * NV + k] = bb[k];
          zs[q * NV + k] = c[k];
        }
      } else {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          const bool ok = i + k < n;
          xs[q * NV + k] = ok ? px[i + k] : (T)0;
          ys[q * NV + k] = ok ? py[i + k] : (T)0;
          zs[q * NV + k] = ok ? pz[i + k] : (T)0;
        }
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int64_t i = chunk_index<T, kScatterThreads>(false, c0, j);
      const bool ok = i < n;
      xs[j] = ok ? px[i] : (T)0;
      ys[j] = ok ? py[i] : (T)0;
      zs[j] = ok ? pz[i] : (T)0;
    }
  }
  int key[PER];
  unsigned rank[PER];
  if (LDSHIST) __syncthreads();              // lcnt cleared
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t i = chunk_index<T, kScatterThreads>(vec, c0, j);
    key[j] = i < n ? locate<T, SCH>(xs[j], ys[j], zs[j], g, m, bg).key : -1;
    if (LDSHIST) rank[j] = key[j] >= 0 ? rank_add(lcnt, key[j]) : 0u;
    else rank[j] = key[j] >= 0 ? rank_add(cursor, key[j]) : 0u;
  }
  if constexpr (STAGE) {
    scatter_stage_chunk<T, false>(lcnt, lbase, srec, skey, wa, wb, cursor, bg, key, rank, xs, ys, zs, c0, n, vec, out,
                                  inv);
    return;
  }
  if (LDSHIST) {
    __syncthreads();
    // lane t reserves tiles t, t + 1024, ... (at most kStageRun of them when
    // the histogram fits in LDS), every reservation issued before any result
    // is used
    unsigned cv[kStageRun], rv[kStageRun];
#pragma unroll
    for (int q = 0; q < kStageRun; ++q) {
      const int k = (int)threadIdx.x + q * kScatterThreads;
      cv[q] = k <= bg.K ? lcnt[k] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kStageRun; ++q)
      rv[q] = cv[q] ? atomicAdd(&cursor[threadIdx.x + q * kScatterThreads], cv[q]) : 0u;
#pragma unroll
    for (int q = 0; q < kStageRun; ++q)
      if (cv[q]) lbase[threadIdx.x + q * kScatterThreads] = rv[q];
    __syncthreads();
  }
  unsigned dv[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) dv[j] = key[j] < 0 ? 0u : LDSHIST ? lbase[key[j]] + rank[j] : rank[j];
  if (vec && c0 + CH <= n) {
    // a whole chunk: no branches between the stores, so none waits for the last
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < PER; ++j) out.st(dv[j], P4{xs[j], ys[j], zs[j]});
    if (!inv) return;
    struct alignas(NV * sizeof(unsigned)) U { unsigned v[NV]; };
#pragma unroll
    for (int q = 0; q < PER / NV; ++q) {
      U u;
#pragma unroll
      for (int k = 0; k < NV; ++k) u.v[k] = dv[q * NV + k];
      *reinterpret_cast<U*>(inv + chunk_index<T, kScatterThreads>(true, c0, q * NV)) = u;
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if (key[j] < 0) continue;
    const int64_t i = chunk_index<T, kScatterThreads>(vec, c0, j);
    out.st(dv[j], P4{xs[j], ys[j], zs[j]});
    if (inv) inv[i] = dv[j];
  }
}

// Staged scatter of whole chunks with the next chunk's positions in flight:
// workgroup w takes chunks w, w + G, ... (G = gridDim.x, a multiple of kXcd,
// one workgroup per CU), and loads chunk c + G while chunk c is ranked,
// staged and stored.  One element whose positions are 16-byte aligned; the
// chunks are the first nfull (whole) ones.
template <typename T, int SCH, bool SOA>
__global__ __launch_bounds__(kScatterThreads) void k_bin_scatter_pipe(ElemBatch eb, const Geometry* geo, size_t stride,
                                                                      char* slot_base, size_t bins_off,
                                                                      char* sorted_base, size_t sorted_stride,
                                                                      size_t inv_off, MeshDims m, BinGeom bg,
                                                                      int nchunk, int nfull, SortedOut<T> so) {
  extern __shared__ unsigned lds[];
  __shared__ unsigned wa[16], wb[16];
  constexpr int PER = chunk_per<T, kScatterThreads>();
  constexpr int NV = Vec16<T>::n;
  constexpr int64_t CH = scatter_chunk<T>();
  using P4 = Rec<T>;
  using V = typename Vec16<T>::type;
  const int b = blockIdx.y;
  const dks_particle_set e = eb.at(b);
  const int64_t n = eb.n(e);
  int c = blockIdx.x;
  if (c >= nfull) return;                    // whole workgroup
  unsigned* lcnt = lds;
  unsigned* lbase = lds + (bg.K + 1);
  P4* srec = reinterpret_cast<P4*>(lds + 2 * (bg.K + 1));
  unsigned short* skey = reinterpret_cast<unsigned short*>(srec + CH);
  const T* px = (const T*)e.x;
  const T* py = (const T*)e.y;
  const T* pz = (const T*)e.z;
  const Geometry gcopy = *geo_of(geo, stride, b);
  const Geometry* g = &gcopy;
  BinState st = bin_state(slot_base, stride, bins_off, b, bg.K);
  const Recs<T, SOA> out = recs_of<T, SOA>(sorted_base, sorted_stride, b, so);
  unsigned* inv = SOA ? so.inv : reinterpret_cast<unsigned*>(sorted_base + (size_t)b * sorted_stride + inv_off);
  auto load = [&](int ch, T (&x)[PER], T (&y)[PER], T (&z)[PER]) {
#pragma unroll
    for (int q = 0; q < PER / NV; ++q) {
      const int64_t i = chunk_index<T, kScatterThreads>(true, (int64_t)ch * CH, q * NV);
      const V a = ld_stream(px + i), bb = ld_stream(py + i), cc = ld_stream(pz + i);
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        x[q * NV + k] = a[k];
        y[q * NV + k] = bb[k];
        z[q * NV + k] = cc[k];
      }
    }
  };
  for (int k = threadIdx.x; k <= bg.K; k += kScatterThreads) lcnt[k] = 0;
  T xs[PER], ys[PER], zs[PER];
  load(c, xs, ys, zs);
  for (;;) {
    unsigned* cursor = st.xcursor + (int)(((int64_t)b * nchunk + c) % kXcd) * (bg.K + 1);
    __syncthreads();                         // lcnt cleared, the previous chunk's records read
    int key[PER];
    unsigned rank[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      key[j] = locate<T, SCH>(xs[j], ys[j], zs[j], g, m, bg).key;
      rank[j] = rank_add(lcnt, key[j]);
    }
    // the next chunk, loaded once the reservations are back (the last chunk
    // re-reads itself, so no load is conditional)
    const int cn = c + (int)gridDim.x;
    const bool more = cn < nfull;
    T nxs[PER], nys[PER], nzs[PER];
    scatter_stage_chunk<T, true>(lcnt, lbase, srec, skey, wa, wb, cursor, bg, key, rank, xs, ys, zs,
                                 (int64_t)c * CH, n, true, out, inv,
                                 [&]() { load(more ? cn : c, nxs, nys, nzs); });
    if (!more) break;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      xs[j] = nxs[j];
      ys[j] = nys[j];
      zs[j] = nzs[j];
    }
    c = cn;
  }
}

// Work item t -> (tile, first particle, one past the last).
// The range is clamped to the binned-particle buffer (max_np records).
__device__ __forceinline__ void decode_item(const BinState& st, const BinGeom& bg, unsigned t, int* tile,
                                            unsigned* start, unsigned* end) {
  int lo = 0, hi = bg.K + 1;   // item_off[lo] <= t < item_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (st.item_off[mid] <= t) lo = mid;
    else hi = mid;
  }
  *tile = lo;
  const unsigned e = min(min(st.offset[lo] + (t - st.item_off[lo]) * (unsigned)bg.item + (unsigned)bg.item,
                             st.offset[lo + 1]),
                         bg.max_np);
  *start = min(st.offset[lo] + (t - st.item_off[lo]) * (unsigned)bg.item, e);
  *end = e;
}

// ---------------------------------------------------------------------------
// deposit: LDS-privatised accumulation per work item, then merge.
// ---------------------------------------------------------------------------
// iacc (the order-independent deposit): instead of adding each work item's
// sum to W in floating point, add the fixed-point sum itself to a per-node
// integer total (FP32: one 64-bit word, which holds 2^32 particles' weights;
// FP64: two words, low and high, with the carry out of the low one), so that
// the totals, and W formed from them afterwards, do not depend on the order
// of the additions.
template <typename T>
__device__ __forceinline__ void add_fixed_total(unsigned long long* node, unsigned long long fv) {
  if constexpr (sizeof(T) == 4) {
    atomicAdd(node, fv);
  } else {
    const unsigned long long old = atomicAdd(node, fv);
    if (old + fv < old) atomicAdd(node + 1, 1ull);
  }
}

template <typename T, int SCH, bool SOA>
__global__ __launch_bounds__(kDepositThreads) void k_deposit_binned(const Geometry* geo, size_t stride, char* slot_base,
                                                        size_t bins_off, const char* sorted_base,
                                                        size_t sorted_stride, T* W, size_t w_stride, MeshDims m,
                                                        BinGeom bg, SortedOut<T> so,
                                                        unsigned long long* iacc, size_t ia_stride) {
  constexpr int A = acc_edge<SCH>(), NN = A * A * A, WD = Scheme<SCH>::width;
  __shared__ unsigned long long acc[NN];
  using P4 = Rec<T>;
  const int b = blockIdx.y;
  const Geometry gcopy = *geo_of(geo, stride, b);   // private copy: not reloaded after each store
  const Geometry* g = &gcopy;
  BinState st = bin_state(slot_base, stride, bins_off, b, bg.K);
  const Recs<T, SOA> part = recs_of<T, SOA>(const_cast<char*>(sorted_base), sorted_stride, b, so);
  T* w = W + (size_t)b * w_stride;
  unsigned long long* ia = iacc ? iacc + (size_t)b * ia_stride : nullptr;
  const unsigned nitems = min(st.misc[0], bg.max_items);
  for (unsigned t = blockIdx.x; t < nitems; t += gridDim.x) {
    int tile;
    unsigned s0, s1;
    decode_item(st, bg, t, &tile, &s0, &s1);
    if (tile == bg.K) continue;                      // outside particles deposit nothing
    const int tx = tile % bg.tx, ty = (tile / bg.tx) % bg.ty, tz = tile / (bg.tx * bg.ty);
    // first node of the accumulator (the tile's first stencil node)
    const int bx = tx * kTile + Scheme<SCH>::lo, by = ty * kTile + Scheme<SCH>::lo, bz = tz * kTile + Scheme<SCH>::lo;
    for (int e = threadIdx.x; e < NN; e += blockDim.x) acc[e] = 0ull;
    __syncthreads();
    // The next group of records is loaded while this one is deposited (the
    // loop issues no other vector-memory operation, so waiting for them is
    // exact).
    // Loads past the item's end re-read its last record (s1 > s0 here), so
    // that no load is conditional: a conditional one makes the compiler wait
    // for every load in flight before the next use.
    P4 pr[kUnrollDeposit], nx[kUnrollDeposit];
    if (s1 > s0) {
#pragma unroll
      for (int u = 0; u < kUnrollDeposit; ++u) pr[u] = part.ld(min(s0 + threadIdx.x + u * blockDim.x, s1 - 1));
    }
    for (unsigned i0 = s0 + threadIdx.x; i0 < s1; i0 += kUnrollDeposit * blockDim.x) {
#pragma unroll
      for (int u = 0; u < kUnrollDeposit; ++u) nx[u] = part.ld(min(i0 + (kUnrollDeposit + u) * blockDim.x, s1 - 1));
#pragma unroll
      for (int u = 0; u < kUnrollDeposit; ++u) {
        if (i0 + u * blockDim.x >= s1) break;
        const P4 p = pr[u];
        const Cell<T, SCH> c = locate<T, SCH>(p.x, p.y, p.z, g, m, bg);
        T wxs[WD];
#pragma unroll
        for (int k = 0; k < WD; ++k) wxs[k] = c.wx[k] * Fixed<T>::scale;   // exact scaling
        unsigned long long* a = acc + ((c.bz - bz) * A + (c.by - by)) * A + (c.bx - bx);
#pragma unroll
        for (int kz = 0; kz < WD; ++kz)
#pragma unroll
          for (int ky = 0; ky < WD; ++ky) {
            const T zy = c.wz[kz] * c.wy[ky];
#pragma unroll
            for (int kx = 0; kx < WD; ++kx) atomicAdd(a + (kz * A + ky) * A + kx, Fixed<T>::to(zy * wxs[kx]));
          }
      }
#pragma unroll
      for (int u = 0; u < kUnrollDeposit; ++u) pr[u] = nx[u];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NN; e += blockDim.x) {
      const unsigned long long fv = acc[e];
      if (fv != 0ull) {
        const int ex = e % A, ey = (e / A) % A, ez = e / (A * A);
        const int x = bx + ex, y = by + ey, z = bz + ez;
        if (x >= 0 && y >= 0 && z >= 0 && x < m.nx && y < m.ny && z < m.nz) {
          const size_t node = ((size_t)z * m.ny + y) * m.nx + x;
          if (ia) add_fixed_total<T>(ia + node * (sizeof(T) == 4 ? 1 : 2), fv);
          else unsafeAtomicAdd(&w[node], Fixed<T>::from(fv));
        }
      }
    }
    __syncthreads();
  }
}

// The order-independent deposit's totals -> W: one conversion of each exact
// integer total (FP64: high word times 2^64 plus the low word, in units of
// the fixed-point scale).
template <typename T>
__global__ __launch_bounds__(256) void k_fixed_to_weights(const unsigned long long* __restrict__ iacc,
                                                          size_t ia_stride, T* __restrict__ W, size_t w_stride,
                                                          size_t nmesh) {
  const unsigned long long* ia = iacc + (size_t)blockIdx.y * ia_stride;
  T* w = W + (size_t)blockIdx.y * w_stride;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nmesh; i += (size_t)gridDim.x * blockDim.x) {
    if constexpr (sizeof(T) == 4) {
      w[i] = Fixed<T>::from(ia[i]);
    } else {
      const unsigned long long lo = ia[2 * i], hi = ia[2 * i + 1];
      w[i] = (double)hi * 32768.0 + Fixed<T>::from(lo);     // 2^64 * 2^-49 = 2^15
    }
  }
}

// ---------------------------------------------------------------------------
// gather with the central-difference field formed on the fly from staged phi
// (FP64, and FP32 TSC; FP32 CIC and NGP use k_gather_binned_field below).
// ---------------------------------------------------------------------------
// SOA (tile-ordered step of a single solve): the records are the caller's
// position arrays so.x/y/z, and the field of record i goes to
// so.ex/ey/ez[i] (no unsort follows); otherwise the field overwrites the
// record in the particle scratch.
template <typename T, int SCH, bool SOA>
__global__ __launch_bounds__(kGatherThreads) void k_gather_binned(const Geometry* geo, size_t stride, char* slot_base,
                                                       size_t bins_off, char* sorted_base, size_t sorted_stride,
                                                       const T* __restrict__ phi_ext, size_t phi_stride,
                                                       MeshDims m, BinGeom bg, SortedOut<T> so) {
  constexpr int A = apron_edge<SCH>(), NA = A * A * A, WD = Scheme<SCH>::width;
  __shared__ T ph[NA];
  using P4 = Rec<T>;
  const int b = blockIdx.y;
  const Geometry gcopy = *geo_of(geo, stride, b);   // private copy: not reloaded after each store
  const Geometry* g = &gcopy;
  BinState st = bin_state(slot_base, stride, bins_off, b, bg.K);
  const Recs<T, SOA> part = recs_of<T, SOA>(sorted_base, sorted_stride, b, so);
  const T* phi = phi_ext + (size_t)b * phi_stride;
  const T cx = Geo<T>::grad(g, 0), cy = Geo<T>::grad(g, 1), cz = Geo<T>::grad(g, 2);
  const int nx2 = m.nx + 2, ny2 = m.ny + 2, nz2 = m.nz + 2;
  const unsigned nitems = min(st.misc[0], bg.max_items);
  for (unsigned t = blockIdx.x; t < nitems; t += gridDim.x) {
    int tile;
    unsigned s0, s1;
    decode_item(st, bg, t, &tile, &s0, &s1);
    if (tile == bg.K) {
      for (unsigned i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
        if constexpr (SOA) {
          so.ex[i] = (T)0;
          so.ey[i] = (T)0;
          so.ez[i] = (T)0;
        } else {
          part.st(i, P4{(T)0, (T)0, (T)0});
        }
      }
      continue;
    }
    const int tx = tile % bg.tx, ty = (tile / bg.tx) % bg.ty, tz = tile / (bg.tx * bg.ty);
    // first stencil node of the tile; staged value e holds node b? - 1 + e,
    // which is phi_ext index b? + e (phi_ext index = node + 1)
    const int bx = tx * kTile + Scheme<SCH>::lo, by = ty * kTile + Scheme<SCH>::lo, bz = tz * kTile + Scheme<SCH>::lo;
    for (int e = threadIdx.x; e < NA; e += blockDim.x) {
      const int ex = e % A, ey = (e / A) % A, ez = e / (A * A);
      const int x = bx + ex, y = by + ey, z = bz + ez;
      const bool in_yz = y >= 0 && z >= 0 && y < ny2 && z < nz2;
      const T* row = phi + ((size_t)z * ny2 + y) * nx2;
      ph[e] = (in_yz && x >= 0 && x < nx2) ? row[x] : (T)0;
    }
    __syncthreads();
    // Unconditional loads (past the item's end they re-read its last record;
    // s1 > s0 inside the loop).  Loading the next group during this one's
    // work (tried) needs registers that halve the occupancy: 794 us, not 687.
    for (unsigned i0 = s0 + threadIdx.x; i0 < s1; i0 += kUnrollGather * blockDim.x) {
      P4 pr[kUnrollGather];
#pragma unroll
      for (int u = 0; u < kUnrollGather; ++u) pr[u] = part.ld(min(i0 + u * blockDim.x, s1 - 1));
#pragma unroll
      for (int u = 0; u < kUnrollGather; ++u) {
        const unsigned i = i0 + u * blockDim.x;
        if (i >= s1) break;
        const P4 p = pr[u];
        const Cell<T, SCH> c = locate<T, SCH>(p.x, p.y, p.z, g, m, bg);
        // staged index of the first stencil node: (node - tile's first node) + 1 per axis
        const int o_idx = ((c.bz - bz + 1) * A + (c.by - by + 1)) * A + (c.bx - bx + 1);
        T ax = 0, ay = 0, az = 0;
        if constexpr (SCH == kSchemeCIC) {
          const T* o = ph + o_idx;
          const T* wx = c.wx;
          const T* wy = c.wy;
          const T* wz = c.wz;
          // The 32 distinct nodes the eight central differences use: four x
          // values per (y, z) corner row, and the y and z neighbours beyond the
          // corner cube.
          T r[2][2][4], ym[2][2], yp[2][2], zm[2][2], zp[2][2];
#pragma unroll
          for (int kz = 0; kz < 2; ++kz)
#pragma unroll
            for (int ky = 0; ky < 2; ++ky)
#pragma unroll
              for (int k = 0; k < 4; ++k) r[kz][ky][k] = o[(kz * A + ky) * A + k - 1];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int kx = 0; kx < 2; ++kx) {
              ym[a][kx] = o[(a * A - 1) * A + kx];         // (x + kx, y - 1, z + a)
              yp[a][kx] = o[(a * A + 2) * A + kx];         // (x + kx, y + 2, z + a)
              zm[a][kx] = o[(-A + a) * A + kx];            // (x + kx, y + a, z - 1)
              zp[a][kx] = o[(2 * A + a) * A + kx];         // (x + kx, y + a, z + 2)
            }
          // E_d = c_d * sum over the eight corners of weight * (phi(+1) - phi(-1)),
          // the coefficient applied once at the end.
#pragma unroll
          for (int kz = 0; kz < 2; ++kz)
#pragma unroll
            for (int ky = 0; ky < 2; ++ky) {
              const T d0 = r[kz][ky][2] - r[kz][ky][0], d1 = r[kz][ky][3] - r[kz][ky][1];
              ax += wz[kz] * wy[ky] * (wx[0] * d0 + wx[1] * d1);
            }
#pragma unroll
          for (int kz = 0; kz < 2; ++kz)
#pragma unroll
            for (int kx = 0; kx < 2; ++kx) {
              const T d0 = r[kz][1][kx + 1] - ym[kz][kx], d1 = yp[kz][kx] - r[kz][0][kx + 1];
              ay += wz[kz] * wx[kx] * (wy[0] * d0 + wy[1] * d1);
            }
#pragma unroll
          for (int ky = 0; ky < 2; ++ky)
#pragma unroll
            for (int kx = 0; kx < 2; ++kx) {
              const T d0 = r[1][ky][kx + 1] - zm[ky][kx], d1 = zp[ky][kx] - r[0][ky][kx + 1];
              az += wy[ky] * wx[kx] * (wz[0] * d0 + wz[1] * d1);
            }
        } else {
          const T* o = ph + o_idx;
          // every stencil node: weight * (phi(+1) - phi(-1)) per axis
#pragma unroll
          for (int kz = 0; kz < WD; ++kz)
#pragma unroll
            for (int ky = 0; ky < WD; ++ky)
#pragma unroll
              for (int kx = 0; kx < WD; ++kx) {
                const T* q = o + (kz * A + ky) * A + kx;
                const T wgt = c.wz[kz] * c.wy[ky] * c.wx[kx];
                ax += wgt * (q[1] - q[-1]);
                ay += wgt * (q[A] - q[-A]);
                az += wgt * (q[A * A] - q[-A * A]);
              }
        }
        if constexpr (SOA) {
          so.ex[i] = ax * cx;
          so.ey[i] = ay * cy;
          so.ez[i] = az * cz;
        } else {
          part.st(i, P4{ax * cx, ay * cy, az * cz});
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// FP32 gather from the field differences at the tile's nodes.  A workgroup
// first forms the central differences (phi(+1) - phi(-1) per axis) at the
// E^3 nodes a 16^3-node tile's particles touch (E = 16 + width - 1: 17 CIC,
// 16 NGP, 18 TSC), straight from phi (the reads of neighbouring nodes hit
// L2), as one 16-byte LDS entry per node; a CIC particle then needs 8
// entries and 36 multiply-adds (trilinear weights of its cell times the
// node differences), against 32 node values and about twice the arithmetic
// when the differences are formed per particle.  The entries take 77 KB
// (CIC) or 64 KB (NGP): two 1024-lane workgroups per CU.  (TSC would need
// 91 KB, one workgroup per CU; it keeps k_gather_binned.)
// ---------------------------------------------------------------------------
template <int SCH> constexpr int field_edge() { return acc_edge<SCH>(); }
template <int SCH> constexpr size_t field_lds_bytes() {
  return (size_t)field_edge<SCH>() * field_edge<SCH>() * field_edge<SCH>() * sizeof(float4);
}
template <int SCH, bool SOA>
__global__ __launch_bounds__(1024) void k_gather_binned_field(const Geometry* geo, size_t stride, char* slot_base,
                                                              size_t bins_off, char* sorted_base,
                                                              size_t sorted_stride, const float* __restrict__ phi_ext,
                                                              size_t phi_stride, MeshDims m, BinGeom bg,
                                                              SortedOut<float> so) {
  constexpr int E = field_edge<SCH>(), WD = Scheme<SCH>::width;
  __shared__ float4 ef[E * E * E];
  using P4 = Rec<float>;
  const int b = blockIdx.y;
  const Geometry gcopy = *geo_of(geo, stride, b);   // private copy: not reloaded after each store
  const Geometry* g = &gcopy;
  BinState st = bin_state(slot_base, stride, bins_off, b, bg.K);
  const Recs<float, SOA> part = recs_of<float, SOA>(sorted_base, sorted_stride, b, so);
  const float* phi = phi_ext + (size_t)b * phi_stride;
  const float cx = Geo<float>::grad(g, 0), cy = Geo<float>::grad(g, 1), cz = Geo<float>::grad(g, 2);
  const int nx2 = m.nx + 2, ny2 = m.ny + 2, nz2 = m.nz + 2;
  const unsigned nitems = min(st.misc[0], bg.max_items);
  for (unsigned t = blockIdx.x; t < nitems; t += gridDim.x) {
    int tile;
    unsigned s0, s1;
    decode_item(st, bg, t, &tile, &s0, &s1);
    if (tile == bg.K) {
      for (unsigned i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
        if constexpr (SOA) {
          so.ex[i] = 0.f;
          so.ey[i] = 0.f;
          so.ez[i] = 0.f;
        } else {
          part.st(i, P4{0.f, 0.f, 0.f});
        }
      }
      continue;
    }
    const int tx = tile % bg.tx, ty = (tile / bg.tx) % bg.ty, tz = tile / (bg.tx * bg.ty);
    // entry e holds node (bx, by, bz) + (e % E, e / E % E, e / E^2), the
    // tile's first stencil node onwards; its phi_ext index is node + 1 per
    // axis, and phi outside phi_ext reads as 0
    const int bx = tx * kTile + Scheme<SCH>::lo, by = ty * kTile + Scheme<SCH>::lo, bz = tz * kTile + Scheme<SCH>::lo;
    for (int e = threadIdx.x; e < E * E * E; e += blockDim.x) {
      const int x = bx + e % E + 1, y = by + (e / E) % E + 1, z = bz + e / (E * E) + 1;
      auto at = [&](int xx, int yy, int zz) {
        return (xx >= 0 && yy >= 0 && zz >= 0 && xx < nx2 && yy < ny2 && zz < nz2)
                   ? phi[((size_t)zz * ny2 + yy) * nx2 + xx]
                   : 0.f;
      };
      ef[e] = make_float4(at(x + 1, y, z) - at(x - 1, y, z), at(x, y + 1, z) - at(x, y - 1, z),
                          at(x, y, z + 1) - at(x, y, z - 1), 0.f);
    }
    __syncthreads();
    // Unconditional loads (past the item's end they re-read its last record;
    // s1 > s0 inside the loop).
    for (unsigned i0 = s0 + threadIdx.x; i0 < s1; i0 += kUnrollGather * blockDim.x) {
      P4 pr[kUnrollGather];
#pragma unroll
      for (int u = 0; u < kUnrollGather; ++u) pr[u] = part.ld(min(i0 + u * blockDim.x, s1 - 1));
#pragma unroll
      for (int u = 0; u < kUnrollGather; ++u) {
        const unsigned i = i0 + u * blockDim.x;
        if (i >= s1) break;
        const P4 p = pr[u];
        const Cell<float, SCH> c = locate<float, SCH>(p.x, p.y, p.z, g, m, bg);
        const float4* o = ef + ((c.bz - bz) * E + (c.by - by)) * E + (c.bx - bx);
        float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
        for (int kz = 0; kz < WD; ++kz)
#pragma unroll
          for (int ky = 0; ky < WD; ++ky) {
            const float w = c.wz[kz] * c.wy[ky];
            float rx = 0.f, ry = 0.f, rz = 0.f;
#pragma unroll
            for (int kx = 0; kx < WD; ++kx) {
              const float4 d = o[(kz * E + ky) * E + kx];
              rx += c.wx[kx] * d.x;
              ry += c.wx[kx] * d.y;
              rz += c.wx[kx] * d.z;
            }
            ax += w * rx;
            ay += w * ry;
            az += w * rz;
          }
        if constexpr (SOA) {
          so.ex[i] = ax * cx;
          so.ey[i] = ay * cy;
          so.ez[i] = az * cz;
        } else {
          part.st(i, P4{ax * cx, ay * cy, az * cz});
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// unsort: E at the particles in their original order.  One workgroup per
// scatter chunk, every load of the chunk issued before any store: the
// chunk's records sit in one short segment per touched tile, so the
// scattered record reads share cache lines within the workgroup.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kUnsortThreads) void k_unsort(ElemBatch eb, const char* sorted_base,
                                                            size_t sorted_stride, size_t inv_off) {
  constexpr int PER = chunk_per<T, kUnsortThreads>();
  constexpr int NV = Vec16<T>::n;
  constexpr int64_t CH = scatter_chunk<T>();
  using P4 = Rec<T>;
  using V = typename Vec16<T>::type;
  const int b = blockIdx.y;
  const dks_particle_set s = eb.at(b);
  const int64_t n = eb.n(s);
  const int64_t c0 = (int64_t)blockIdx.x * CH;
  if (c0 >= n) return;
  const P4* part = reinterpret_cast<const P4*>(sorted_base + (size_t)b * sorted_stride);
  const unsigned* inv = reinterpret_cast<const unsigned*>(sorted_base + (size_t)b * sorted_stride + inv_off);
  T* qx = (T*)s.Ex;
  T* qy = (T*)s.Ey;
  T* qz = (T*)s.Ez;
  const bool vec = aligned16(qx + c0, qy + c0, qz + c0);
  if (vec && c0 + CH <= n) {
    // A whole chunk in the vector layout: straight-line code, so that every
    // load is issued before the first wait and the stores go out back to
    // back (a branch between them would make each wait for the last).
    typedef unsigned UV __attribute__((ext_vector_type(NV)));
    unsigned src[PER];
#pragma unroll
    for (int q = 0; q < PER / NV; ++q) {
      const int64_t i = chunk_index<T, kUnsortThreads>(true, c0, q * NV);
      const UV v = __builtin_nontemporal_load((const __attribute__((address_space(1))) UV*)(inv + i));
#pragma unroll
      for (int k = 0; k < NV; ++k) src[q * NV + k] = v[k];
    }
    V ax[PER / NV], ay[PER / NV], az[PER / NV];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const P4 r = part[src[j]];
      ax[j / NV][j % NV] = r.x;
      ay[j / NV][j % NV] = r.y;
      az[j / NV][j % NV] = r.z;
    }
#pragma unroll
    for (int q = 0; q < PER / NV; ++q) {
      const int64_t i = chunk_index<T, kUnsortThreads>(true, c0, q * NV);
      st_stream(qx + i, ax[q]);
      st_stream(qy + i, ay[q]);
      st_stream(qz + i, az[q]);
    }
    return;
  }
  unsigned src[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t i = chunk_index<T, kUnsortThreads>(vec, c0, j);
    src[j] = i < n ? __builtin_nontemporal_load(inv + i) : 0u;
  }
  T ex[PER], ey[PER], ez[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const P4 r = part[src[j]];
    ex[j] = r.x;
    ey[j] = r.y;
    ez[j] = r.z;
  }
  if (vec) {
#pragma unroll
    for (int q = 0; q < PER / NV; ++q) {
      const int64_t i = chunk_index<T, kUnsortThreads>(true, c0, q * NV);
      if (i + NV <= n) {
        V a, bb, c;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          a[k] = ex[q * NV + k];
          bb[k] = ey[q * NV + k];
          c[k] = ez[q * NV + k];
        }
        st_stream(qx + i, a);
        st_stream(qy + i, bb);
        st_stream(qz + i, c);
      } else {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
          if (i + k < n) {
            qx[i + k] = ex[q * NV + k];
            qy[i + k] = ey[q * NV + k];
            qz[i + k] = ez[q * NV + k];
          }
        }
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int64_t i = chunk_index<T, kUnsortThreads>(false, c0, j);
      if (i < n) {
        qx[i] = ex[j];
        qy[i] = ey[j];
        qz[i] = ez[j];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <typename T> static SortedOut<T> sorted_out(void* const* soa) {
  if (!soa) return SortedOut<T>{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  return SortedOut<T>{(T*)soa[0], (T*)soa[1], (T*)soa[2], (T*)soa[3], (T*)soa[4], (T*)soa[5], (unsigned*)soa[6]};
}

// f(scheme constant, SOA constant)
template <class F> static void with_scheme_soa(int scheme, bool soa, F&& f) {
  with_scheme(scheme, [&](auto sc) {
    if (soa) f(sc, std::true_type{});
    else f(sc, std::false_type{});
  });
}

template <typename T>
hipError_t launch_bin_count(const ElemBatch& eb, int batch, const Geometry* geo, size_t stride, char* slot_base, size_t bins_off,
                            const MeshDims& m, const BinGeom& bg, int nblk, hipStream_t s) {
  (void)nblk;
  if (eb.max_np == 0) return hipSuccess;
  const int64_t nchunk = (eb.max_np + scatter_chunk<T>() - 1) / scatter_chunk<T>();
  // a multiple of kXcd, so every chunk a workgroup walks is in one XCD group
  const unsigned grid = (unsigned)std::min<int64_t>(1024, (nchunk + kXcd - 1) / kXcd * kXcd);
  const bool lh = bg.lds_hist != 0;
  const size_t lds = lh ? (size_t)(bg.K + 1) * sizeof(unsigned) : 0;
  with_scheme(bg.scheme, [&](auto sc) {
    constexpr int SCH = decltype(sc)::value;
    if (lh)
      hipLaunchKernelGGL((k_bin_count<T, true, SCH>), dim3(grid, batch), dim3(256), lds, s, eb, geo, stride,
                         slot_base, bins_off, m, bg, (int)nchunk);
    else
      hipLaunchKernelGGL((k_bin_count<T, false, SCH>), dim3(grid, batch), dim3(256), 0, s, eb, geo, stride,
                         slot_base, bins_off, m, bg, (int)nchunk);
  });
  return hipGetLastError();
}

hipError_t launch_bin_scan(const Geometry* geo, size_t stride, char* slot_base, size_t bins_off, const BinGeom& bg,
                           const ElemBatch& eb, int batch, hipStream_t s) {
  hipLaunchKernelGGL(k_bin_scan, dim3(batch), dim3(1024), 0, s, geo, stride, slot_base, bins_off, bg, eb);
  return hipGetLastError();
}

// Compute units of the current device (cached per device).
static int compute_units() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    cache[dev] = v;
  }
  return cache[dev];
}

template <typename T>
hipError_t launch_bin_scatter(const ElemBatch& eb, int batch, const Geometry* geo, size_t stride, char* slot_base, size_t bins_off,
                              char* sorted_base, size_t sorted_stride, size_t inv_off, const MeshDims& m,
                              const BinGeom& bg, int nblk, void* const* soa, hipStream_t s) {
  (void)nblk;
  if (eb.max_np == 0) return hipSuccess;
  if (soa && batch != 1) return hipErrorInvalidValue;
  const SortedOut<T> so = sorted_out<T>(soa);
  const int64_t ch = scatter_chunk<T>();
  const unsigned nchunk = (unsigned)((eb.max_np + ch - 1) / ch);
  const bool lh = bg.lds_hist != 0;
  // 256 bytes left for the static scan scratch
  const bool stage = lh && scatter_stage_lds<T>(bg.K) + 256 <= kLdsPerWorkgroup &&
                     bg.K + 1 <= kStageRun * kScatterThreads;
  const size_t lds = stage ? scatter_stage_lds<T>(bg.K) : lh ? 2 * (size_t)(bg.K + 1) * sizeof(unsigned) : 0;
  // One element with aligned positions and at least one chunk per CU: the
  // whole chunks go through the pipelined kernel, the partial last chunk (if
  // any) through the one-chunk kernel.
  int nfull = 0, G = 0;
  if (stage && batch == 1 && eb.dev == nullptr) {
    const dks_particle_set& e = eb.local;
    const bool have = e.x && e.y && e.z && (!eb.need_e || (e.Ex && e.Ey && e.Ez));
    const int64_t n = have ? std::min<int64_t>(std::max<int64_t>(e.np, 0), eb.max_np) : 0;
    const bool aligned = ((reinterpret_cast<uintptr_t>(e.x) | reinterpret_cast<uintptr_t>(e.y) |
                           reinterpret_cast<uintptr_t>(e.z)) & 15u) == 0;
    const int cus = compute_units();
    if (aligned && cus > 0 && n / ch >= 2 * cus) {
      nfull = (int)(n / ch);
      G = std::max(kXcd, cus / kXcd * kXcd);
    }
  }
  with_scheme_soa(bg.scheme, soa != nullptr, [&](auto sc, auto sa) {
    constexpr int SCH = decltype(sc)::value;
    constexpr bool SOA = decltype(sa)::value;
    if (nfull > 0) {
      hipLaunchKernelGGL((k_bin_scatter_pipe<T, SCH, SOA>), dim3(G, 1), dim3(kScatterThreads), lds, s, eb, geo, stride,
                         slot_base, bins_off, sorted_base, sorted_stride, inv_off, m, bg, (int)nchunk, nfull, so);
      if ((unsigned)nfull < nchunk)
        hipLaunchKernelGGL((k_bin_scatter<T, true, true, SCH, SOA>), dim3(nchunk - nfull, 1), dim3(kScatterThreads), lds,
                           s, eb, geo, stride, slot_base, bins_off, sorted_base, sorted_stride, inv_off, m, bg,
                           nfull, (int)nchunk, so);
    } else if (stage) {
      hipLaunchKernelGGL((k_bin_scatter<T, true, true, SCH, SOA>), dim3(nchunk, batch), dim3(kScatterThreads), lds, s, eb,
                         geo, stride, slot_base, bins_off, sorted_base, sorted_stride, inv_off, m, bg, 0, (int)nchunk,
                         so);
    } else if (lh) {
      hipLaunchKernelGGL((k_bin_scatter<T, true, false, SCH, SOA>), dim3(nchunk, batch), dim3(kScatterThreads), lds, s,
                         eb, geo, stride, slot_base, bins_off, sorted_base, sorted_stride, inv_off, m, bg, 0,
                         (int)nchunk, so);
    } else {
      hipLaunchKernelGGL((k_bin_scatter<T, false, false, SCH, SOA>), dim3(nchunk, batch), dim3(kScatterThreads), 0, s,
                         eb, geo, stride, slot_base, bins_off, sorted_base, sorted_stride, inv_off, m, bg, 0,
                         (int)nchunk, so);
    }
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_deposit_binned(const Geometry* geo, size_t stride, char* slot_base, size_t bins_off,
                                 const char* sorted_base, size_t sorted_stride, void* W, size_t w_stride,
                                 const MeshDims& m, const BinGeom& bg, int nblk, int batch, void* const* soa,
                                 void* iacc, size_t ia_stride, hipStream_t s) {
  if (soa && batch != 1) return hipErrorInvalidValue;
  const SortedOut<T> so = sorted_out<T>(soa);
  with_scheme_soa(bg.scheme, soa != nullptr, [&](auto sc, auto sa) {
    hipLaunchKernelGGL((k_deposit_binned<T, decltype(sc)::value, decltype(sa)::value>), dim3(nblk, batch),
                       dim3(kDepositThreads), 0, s, geo, stride, slot_base, bins_off, sorted_base, sorted_stride,
                       (T*)W, w_stride, m, bg, so, (unsigned long long*)iacc, ia_stride);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fixed_to_weights(const void* iacc, size_t ia_stride, void* W, size_t w_stride, size_t nmesh,
                                   int batch, hipStream_t s) {
  if (nmesh == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((nmesh + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fixed_to_weights<T>, dim3(blocks, batch), dim3(256), 0, s,
                     (const unsigned long long*)iacc, ia_stride, (T*)W, w_stride, nmesh);
  return hipGetLastError();
}

// soa: NULL, or the caller arrays (x, y, z, Ex, Ey, Ez) of the tile-ordered
// step of one element: the records are x, y, z and the field goes to Ex, Ey, Ez.
template <typename T>
hipError_t launch_gather_binned(const Geometry* geo, size_t stride, char* slot_base, size_t bins_off,
                                char* sorted_base, size_t sorted_stride, const void* phi_ext, size_t phi_stride,
                                const MeshDims& m, const BinGeom& bg, int nblk, int batch, void* const* soa,
                                hipStream_t s) {
  if (soa && batch != 1) return hipErrorInvalidValue;
  const SortedOut<T> so = sorted_out<T>(soa);
  if constexpr (sizeof(T) == 4) {
    // TSC's 91 KB of node differences leave one workgroup per CU, and that
    // gather measured slower (1851 against 1675 us at 256^3 / 1e8) than
    // forming the differences per particle
    if (bg.scheme != kSchemeTSC) {
      const bool ngp = bg.scheme == kSchemeNGP;
      if (soa) {
        if (ngp)
          hipLaunchKernelGGL((k_gather_binned_field<kSchemeNGP, true>), dim3(nblk, batch), dim3(1024), 0, s, geo,
                             stride, slot_base, bins_off, sorted_base, sorted_stride, (const float*)phi_ext,
                             phi_stride, m, bg, so);
        else
          hipLaunchKernelGGL((k_gather_binned_field<kSchemeCIC, true>), dim3(nblk, batch), dim3(1024), 0, s, geo,
                             stride, slot_base, bins_off, sorted_base, sorted_stride, (const float*)phi_ext,
                             phi_stride, m, bg, so);
      } else {
        if (ngp)
          hipLaunchKernelGGL((k_gather_binned_field<kSchemeNGP, false>), dim3(nblk, batch), dim3(1024), 0, s, geo,
                             stride, slot_base, bins_off, sorted_base, sorted_stride, (const float*)phi_ext,
                             phi_stride, m, bg, so);
        else
          hipLaunchKernelGGL((k_gather_binned_field<kSchemeCIC, false>), dim3(nblk, batch), dim3(1024), 0, s, geo,
                             stride, slot_base, bins_off, sorted_base, sorted_stride, (const float*)phi_ext,
                             phi_stride, m, bg, so);
      }
      return hipGetLastError();
    }
  }
  with_scheme_soa(bg.scheme, soa != nullptr, [&](auto sc, auto sa) {
    constexpr int SCH = decltype(sc)::value;
    hipLaunchKernelGGL((k_gather_binned<T, SCH, decltype(sa)::value>), dim3(nblk, batch),
                       dim3(kGatherThreads), 0, s, geo, stride, slot_base, bins_off, sorted_base,
                       sorted_stride, (const T*)phi_ext, phi_stride, m, bg, so);
  });
  return hipGetLastError();
}

template <typename T>
hipError_t launch_unsort(const ElemBatch& eb, int batch, const char* sorted_base, size_t sorted_stride,
                         size_t inv_off, hipStream_t s) {
  if (eb.max_np == 0) return hipSuccess;
  const int64_t ch = scatter_chunk<T>();
  const unsigned nchunk = (unsigned)((eb.max_np + ch - 1) / ch);
  hipLaunchKernelGGL(k_unsort<T>, dim3(nchunk, batch), dim3(kUnsortThreads), 0, s, eb, sorted_base,
                     sorted_stride, inv_off);
  return hipGetLastError();
}

#define DKS_INSTANTIATE(T)                                                                                         \
  template hipError_t launch_bin_count<T>(const ElemBatch&, int, const Geometry*, size_t, char*, size_t, const MeshDims&,            \
                                          const BinGeom&, int, hipStream_t);                                       \
  template hipError_t launch_bin_scatter<T>(const ElemBatch&, int, const Geometry*, size_t, char*, size_t,      \
                                            char*, size_t, size_t, const MeshDims&, const BinGeom&, int,           \
                                            void* const*, hipStream_t);                                            \
  template hipError_t launch_deposit_binned<T>(const Geometry*, size_t, char*, size_t, const char*, size_t, void*, \
                                               size_t, const MeshDims&, const BinGeom&, int, int, void* const*,    \
                                               void*, size_t, hipStream_t);                                        \
  template hipError_t launch_fixed_to_weights<T>(const void*, size_t, void*, size_t, size_t, int, hipStream_t);   \
  template hipError_t launch_gather_binned<T>(const Geometry*, size_t, char*, size_t, char*, size_t,               \
                                              const void*, size_t, const MeshDims&, const BinGeom&, int, int,      \
                                              void* const*, hipStream_t);                                          \
  template hipError_t launch_unsort<T>(const ElemBatch&, int, const char*, size_t, size_t, hipStream_t);
DKS_INSTANTIATE(float)
DKS_INSTANTIATE(double)
#undef DKS_INSTANTIATE

}  // namespace dks
