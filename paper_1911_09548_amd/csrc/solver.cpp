// The stmg C ABI: setup of the space-time hierarchy, device uploads and the
// V-cycle driver (sections 2-4 of the paper; see include/stmg.h).
#include "solver.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <mutex>
#include <new>
#include <numeric>
#include <system_error>
#include <thread>
#include <type_traits>
#include <cstring>

using namespace stmg;

namespace stmg {
void alloc_point(const char *what);
}

namespace {

constexpr int GRAPH_NORM_SLOT = 8192;  // d_scalar[0..8191]: norms of stmg_cycles; [8192]: the graph's
constexpr int FACTOR_WORKERS = 8;      // most threads of the parallel slab factorisations in stmg_setup

thread_local std::string g_err;

// Failure injection (stmg_debug_fail_alloc): allocation points counted
// since the last arming; the armed one (1-based; 0 = off) throws.
std::atomic<int64_t> g_alloc_count{0};
std::atomic<int64_t> g_alloc_fail_at{0};

template <class F>
int guard(F &&fn) {
  try {
    fn();
    return STMG_OK;
  } catch (const StmgError &e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    return STMG_ENOMEM;
  } catch (const std::exception &e) {
    g_err = e.what();
    return STMG_EINVAL;
  }
}

void hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return;
  const int code = (e == hipErrorOutOfMemory) ? STMG_ENOMEM : STMG_EHIP;
  fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

// The stream and rocBLAS handle of setup work in the calling thread: those
// of a worker thread of the parallel slab factorisation, else the handle's.
thread_local hipStream_t tl_setup_stream = nullptr;
thread_local rocblas_handle tl_setup_rb = nullptr;
hipStream_t setup_stream(const stmg_handle *h) { return tl_setup_stream ? tl_setup_stream : h->stream; }
rocblas_handle setup_rb(const stmg_handle *h) { return tl_setup_rb ? tl_setup_rb : h->rb; }

// Handles owned by the server allocate stream-ordered (hipMallocAsync on
// their own stream) so that allocation and release never wait for other
// requests' work; other handles use hipMalloc.
template <typename T>
T *dev_alloc(stmg_handle *h, size_t count) {
  alloc_point("device buffer");
  if (count == 0) count = 1;
  void *p = nullptr;
  if (h->stream_ordered)
    hip_check(hipMallocAsync(&p, count * sizeof(T), h->stream), "hipMallocAsync");
  else
    hip_check(hipMalloc(&p, count * sizeof(T)), "hipMalloc");
  std::lock_guard<std::mutex> lock(h->alloc_mu);
  h->bufs.push_back({p, count * sizeof(T)});
  h->device_bytes += (int64_t)(count * sizeof(T));
  return static_cast<T *>(p);
}

// Copies on the setup stream and waits for that stream only.
template <typename T>
T *dev_upload(stmg_handle *h, const T *src, size_t count) {
  T *p = dev_alloc<T>(h, count);
  if (count) {
    hipStream_t st = setup_stream(h);
    hip_check(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, st), "upload");
    hip_check(hipStreamSynchronize(st), "upload");
  }
  return p;
}

template <typename T>
T *dev_upload(stmg_handle *h, const std::vector<T> &v) {
  return dev_upload(h, v.data(), v.size());
}

// A device buffer that lives only during setup (released on the handle's
// stream for stream-ordered handles, after a synchronisation of the setup
// stream otherwise).
struct DevTemp {
  stmg_handle *h;
  hipStream_t st;
  void *p = nullptr;
  DevTemp(stmg_handle *h_, size_t bytes) : h(h_), st(setup_stream(h_)) {
    alloc_point("device setup temporary");
    if (bytes == 0) bytes = 16;
    if (h->stream_ordered)
      hip_check(hipMallocAsync(&p, bytes, h->stream), "hipMallocAsync");
    else
      hip_check(hipMalloc(&p, bytes), "hipMalloc");
  }
  template <typename T>
  DevTemp(stmg_handle *h_, const std::vector<T> &v) : DevTemp(h_, v.size() * sizeof(T)) {
    if (!v.empty()) {
      hip_check(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st), "upload");
      hip_check(hipStreamSynchronize(st), "upload");
    }
  }
  ~DevTemp() {
    if (!p) return;
    if (h->stream_ordered) {
      (void)hipFreeAsync(p, h->stream);
    } else {
      (void)hipStreamSynchronize(st);
      (void)hipFree(p);
    }
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(p);
  }
  DevTemp(const DevTemp &) = delete;
  DevTemp &operator=(const DevTemp &) = delete;
};

// Set by the host phase from the device_factor option: large factors are
// factored on the GPU; small ones (launch-latency bound there) on the host.
bool dev_factor(const stmg_handle *h) { return h->device_factor_on; }

// Most worker threads of the parallel slab factorisations: FACTOR_WORKERS,
// or the environment's STMG_SETUP_THREADS (1..FACTOR_WORKERS; 1 factors on
// the calling thread's stream only).
int setup_threads_limit() {
  const char *e = getenv("STMG_SETUP_THREADS");
  if (!e || !*e) return FACTOR_WORKERS;
  const int v = atoi(e);
  return v < 1 ? 1 : (v > FACTOR_WORKERS ? FACTOR_WORKERS : v);
}

// Setup progress on stderr (environment STMG_VERBOSE set and not 0).
bool verbose() {
  static const bool v = getenv("STMG_VERBOSE") && getenv("STMG_VERBOSE")[0] != '0';
  return v;
}

// ------------------------------------------------------------- solve plans
void build_plan(stmg_handle *h, const Symbolic &S, DevFactor &D) {
  const int32_t ns = S.ns, H = S.n_heights;
  std::vector<int64_t> uoff(ns, 0);
  int64_t u = 0;
  for (int32_t s = 0; s < ns; ++s) {
    uoff[s] = u;
    u += S.nrows(s);
  }
  D.u_rows = u;
  std::vector<std::vector<int32_t>> kids(ns), by_h(H);
  for (int32_t s = 0; s < ns; ++s) {
    if (S.parent[s] >= 0) kids[S.parent[s]].push_back(s);
    by_h[S.height[s]].push_back(s);
  }
  // forward assembly targets. Per height: first the rows of the supernodes'
  // own columns that receive children's update rows (k_fwd_asm adds them
  // into X), then every update row of those supernodes in row order (their
  // children's contributions are summed by the GEMM epilogue that writes
  // the row); uasm[s] = index of supernode s's first update-row target
  std::vector<AsmTarget> tgt;
  std::vector<int64_t> src;
  std::vector<int64_t> uasm(ns, -1);
  D.h_tgt_off.assign(H + 1, 0);
  D.h_xtgt_end.assign(H, 0);
  D.h_src_off.assign(H + 1, 0);
  D.h_xsrc_end.assign(H, 0);
  std::vector<int32_t> pos(S.n, -1);
  for (int32_t hh = 0; hh < H; ++hh) {
    D.h_tgt_off[hh] = (int64_t)tgt.size();
    D.h_src_off[hh] = (int64_t)src.size();
    std::vector<std::vector<std::vector<int64_t>>> per_s;
    for (int32_t s : by_h[hh]) {
      const int32_t c0 = S.col0[s], w = S.width(s), r = S.nrows(s), m = w + r;
      for (int32_t j = 0; j < w; ++j) pos[c0 + j] = j;
      for (int32_t i = 0; i < r; ++i) pos[S.rows[S.rptr[s] + i]] = w + i;
      std::vector<std::vector<int64_t>> srcs(m);
      for (int32_t ch : kids[s])
        for (int32_t i = 0; i < S.nrows(ch); ++i) srcs[pos[S.rows[S.rptr[ch] + i]]].push_back(uoff[ch] + i);
      for (int32_t t = 0; t < w; ++t) {
        if (srcs[t].empty()) continue;
        tgt.push_back({(int64_t)(c0 + t), (int64_t)src.size()});
        src.insert(src.end(), srcs[t].begin(), srcs[t].end());
      }
      per_s.push_back(std::move(srcs));
    }
    D.h_xtgt_end[hh] = (int64_t)tgt.size();
    D.h_xsrc_end[hh] = (int64_t)src.size();
    for (size_t q = 0; q < by_h[hh].size(); ++q) {
      const int32_t s = by_h[hh][q], w = S.width(s), r = S.nrows(s);
      if (r > 0) uasm[s] = (int64_t)tgt.size();
      for (int32_t t = w; t < w + r; ++t) {
        tgt.push_back({-1 - (uoff[s] + (t - w)), (int64_t)src.size()});
        src.insert(src.end(), per_s[q][t].begin(), per_s[q][t].end());
      }
    }
  }
  D.h_tgt_off[H] = (int64_t)tgt.size();
  D.h_src_off[H] = (int64_t)src.size();
  tgt.push_back({0, (int64_t)src.size()});  // sentinel
  // one forward and one backward GEMM launch per height; one task (supernode,
  // row tile) per 64-row and per 32-row tile
  std::vector<SolveTask> tasks;
  struct Pending {
    size_t off64, off32, n;
    int32_t tiles64, tiles32;
    int64_t rows;
    double nnz, nnz_struct;
    int32_t kmax;
  };
  auto make_pending = [&](int32_t hh, bool fwd) {
    Pending p{tasks.size(), 0, 0, 0, 0, 0, 0.0, 0.0, 0};
    for (int32_t s : by_h[hh]) {
      const int32_t rows = fwd ? S.width(s) + S.nrows(s) : S.width(s);
      for (int32_t t = 0; t < (rows + 63) / 64; ++t) tasks.push_back({s, t});
      p.tiles64 += (rows + 63) / 64;
      p.rows += rows;
      const double w = S.width(s), r = S.nrows(s);
      p.nnz += w * (w + 1) / 2 + r * w;
      p.nnz_struct += (double)S.sn_nnz[s];
      p.kmax = std::max(p.kmax, fwd ? S.width(s) : S.width(s) + S.nrows(s));
    }
    p.n = by_h[hh].size();
    p.off32 = tasks.size();
    for (int32_t s : by_h[hh]) {
      const int32_t rows = fwd ? S.width(s) + S.nrows(s) : S.width(s);
      for (int32_t t = 0; t < (rows + 31) / 32; ++t) tasks.push_back({s, t});
      p.tiles32 += (rows + 31) / 32;
    }
    return p;
  };
  std::vector<Pending> pf(H), pb(H);
  for (int32_t hh = 0; hh < H; ++hh) {
    pf[hh] = make_pending(hh, true);
    pb[hh] = make_pending(hh, false);
  }
  SolveTask *dt = dev_upload(h, tasks);
  AsmTarget *dtg = dev_upload(h, tgt);
  int64_t *dsrc = dev_upload(h, src);
  auto mk = [&](const Pending &p) {
    SolvePlan::Launch L;
    L.nnz = p.nnz;
    L.nnz_struct = p.nnz_struct;
    L.kmax = p.kmax;
    L.n_tasks = (int32_t)p.n;
    L.n_tiles = p.tiles64;
    L.n_tiles32 = p.tiles32;
    L.rows = p.rows;
    L.tasks = dt + p.off64;
    L.tasks32 = dt + p.off32;
    return L;
  };
  for (auto &p : pf) D.fwd.push_back(mk(p));
  for (auto &p : pb) D.bwd.push_back(mk(p));
  // factor metadata
  std::vector<int32_t> m(ns);
  for (int32_t s = 0; s < ns; ++s) m[s] = S.width(s) + S.nrows(s);
  D.f.ns = ns;
  D.f.n = S.n;
  D.f.col0 = dev_upload(h, S.col0);
  D.f.m = dev_upload(h, m);
  D.f.rptr = dev_upload(h, S.rptr);
  D.f.rows = dev_upload(h, S.rows);
  D.f.uoff = dev_upload(h, uoff);
  D.f.uasm = dev_upload(h, uasm);
  D.plan.n_heights = H;
  D.plan.tile_rows = h->opt.gemm_rows;
  D.plan.splitk = h->opt.gemm_splitk;
  D.plan.prof = nullptr;
  D.plan.splitk_ws = nullptr;
  D.plan.splitk_bytes = 0;
  D.plan.h_tgt_off = D.h_tgt_off.data();
  D.plan.h_src_off = D.h_src_off.data();
  D.plan.h_xtgt_end = D.h_xtgt_end.data();
  D.plan.h_xsrc_end = D.h_xsrc_end.data();
  D.plan.tgt = dtg;
  D.plan.src = dsrc;
  D.f.asm_tgt = dtg;
  D.f.asm_src = dsrc;
  D.plan.fwd = D.fwd.data();
  D.plan.bwd = D.bwd.data();
}

// Upload P_s of every supernode (and P_s^T when `transpose`: w x m,
// column-major, which the backward solve then streams with unit stride)
// into `F` with scalar type T; TH is the host FP64 scalar, T may be the FP64
// type or its FP32 counterpart (values rounded to nearest).
inline void narrow(const double &a, double &b) { b = a; }
inline void narrow(const double &a, float &b) { b = (float)a; }
inline void narrow(const cplx &a, cd &b) { b = {a.re, a.im}; }
inline void narrow(const cplx &a, cf &b) { b = {(float)a.re, (float)a.im}; }

template <typename T, typename TH>
void upload_panels(stmg_handle *h, const Symbolic &S, const HostFactor<TH> &F, FactorDev &fd, bool transpose,
                   int64_t &bytes) {
  std::vector<T> P(F.panel.size());
  for (size_t i = 0; i < P.size(); ++i) narrow(F.panel[i], P[i]);
  fd.panel = dev_upload(h, P);
  bytes += (int64_t)(P.size() * sizeof(T));
  fd.panel_t = nullptr;
  if (transpose) {
    std::vector<T> Pt(P.size());
    for (int32_t s = 0; s < S.ns; ++s) {
      const int64_t w = S.width(s), m = w + S.nrows(s), o = F.panel_off[s];
      for (int64_t k = 0; k < w; ++k)
        for (int64_t i = 0; i < m; ++i) Pt[o + k + i * w] = P[o + i + k * m];
    }
    fd.panel_t = dev_upload(h, Pt);
    bytes += (int64_t)(Pt.size() * sizeof(T));
  }
}

// Offsets (shared by both precisions) and the panels each form needs.
template <typename T64, typename T32, typename TH>
void upload_factor(stmg_handle *h, const Symbolic &S, const HostFactor<TH> &F, DevFactor &D, bool transpose,
                   bool need64, bool need32) {
  D.f.panel_off = dev_upload(h, F.panel_off);
  D.h_panel_off = F.panel_off;
  D.f.panel = D.f.panel_t = nullptr;
  D.factor_bytes = 0;
  if (need64) upload_panels<T64>(h, S, F, D.f, transpose, D.factor_bytes);
  D.f32 = D.f;
  D.f32.panel = D.f32.panel_t = nullptr;
  if (need32) upload_panels<T32>(h, S, F, D.f32, transpose, D.factor_bytes);
  std::lock_guard<std::mutex> lock(h->alloc_mu);
  h->factor_bytes += D.factor_bytes;
}

// Numeric factorisation on the device (values `vals` on the pattern the
// front plan was built from), then the panels each form keeps: FP64 (and its
// transpose) and/or FP32 (and its transpose), converted on the device.
template <typename T64, typename T32>
void factor_into(stmg_handle *h, const Symbolic &S, const FrontPlan &fp, const std::vector<T64> &vals,
                 DevFactor &D, bool transpose, bool need64, bool need32) {
  std::vector<int64_t> off;
  factor_layout(S, off);
  const int64_t n = off[S.ns];
  D.h_panel_off = off;
  D.f.panel_off = dev_upload(h, off);
  std::vector<int32_t> width(S.ns);
  for (int32_t s = 0; s < S.ns; ++s) width[s] = S.width(s);
  DevTemp t_width(h, width), t_pos(h, fp.a_pos), t_k(h, fp.a_k), t_rel(h, fp.relpos), t_vals(h, vals);
  DevTemp t_front(h, (size_t)fp.max_m2 * sizeof(T64));
  DevTemp t_arena(h, (size_t)fp.uoff[S.ns] * sizeof(T64));
  DevTemp t_flag(h, sizeof(int32_t));
  DevTemp t_p64(h, need64 ? 0 : (size_t)n * sizeof(T64));
  T64 *p64 = need64 ? dev_alloc<T64>(h, (size_t)n) : t_p64.as<T64>();
  hipStream_t st = setup_stream(h);
  hip_check(hipMemsetAsync(t_flag.p, 0, sizeof(int32_t), st), "memset");
  FrontPlanDev fd;
  fd.a_pos = t_pos.as<int64_t>();
  fd.a_k = t_k.as<int64_t>();
  fd.relpos = t_rel.as<int32_t>();
  factor_device<T64>(S, fp, fd, off, t_vals.as<T64>(), p64, t_front.as<T64>(), t_arena.as<T64>(),
                     t_flag.as<int32_t>(), setup_rb(h), st);
  int32_t bad = 0;
  hip_check(hipMemcpyAsync(&bad, t_flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy");
  hip_check(hipStreamSynchronize(st), "factorisation");
  STMG_REQUIRE(bad == 0, STMG_ENUMERIC, "zero or non-finite pivot in factorisation");
  D.factor_bytes = 0;
  D.f.panel = need64 ? p64 : nullptr;
  D.f.panel_t = nullptr;
  if (need64) {
    D.factor_bytes += n * (int64_t)sizeof(T64);
    if (transpose) {
      T64 *pt = dev_alloc<T64>(h, (size_t)n);
      convert_panels<T64, T64>(p64, nullptr, pt, D.f.panel_off, t_width.as<int32_t>(), S.ns, n, st);
      D.f.panel_t = pt;
      D.factor_bytes += n * (int64_t)sizeof(T64);
    }
  }
  D.f32 = D.f;
  D.f32.panel = D.f32.panel_t = nullptr;
  if (need32) {
    T32 *q = dev_alloc<T32>(h, (size_t)n), *qt = transpose ? dev_alloc<T32>(h, (size_t)n) : nullptr;
    convert_panels<T64, T32>(p64, q, qt, D.f.panel_off, t_width.as<int32_t>(), S.ns, n, st);
    D.f32.panel = q;
    D.f32.panel_t = qt;
    D.factor_bytes += n * (int64_t)sizeof(T32) * (transpose ? 2 : 1);
  }
  hip_check(hipGetLastError(), "kernel launch");
  hip_check(hipStreamSynchronize(st), "factor conversion");
  std::lock_guard<std::mutex> lock(h->alloc_mu);
  h->factor_bytes += D.factor_bytes;
}

// ------------------------------------------------------------ level setup
// Position along the 3D Hilbert curve of a point with 21-bit coordinates
// (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004:
// the axes are turned into the curve's transposed index, whose bits are then
// interleaved).
uint64_t hilbert_key(uint32_t x[3]) {
  constexpr int n = 3, bits = 21;
  const uint32_t top = 1u << (bits - 1);
  for (uint32_t q = top; q > 1; q >>= 1) {
    const uint32_t p = q - 1;
    for (int i = 0; i < n; ++i) {
      if (x[i] & q) {
        x[0] ^= p;
      } else {
        const uint32_t t = (x[0] ^ x[i]) & p;
        x[0] ^= t;
        x[i] ^= t;
      }
    }
  }
  for (int i = 1; i < n; ++i) x[i] ^= x[i - 1];
  uint32_t t = 0;
  for (uint32_t q = top; q > 1; q >>= 1)
    if (x[n - 1] & q) t ^= q - 1;
  for (int i = 0; i < n; ++i) x[i] ^= t;
  uint64_t key = 0;
  for (int b = bits - 1; b >= 0; --b)
    for (int i = 0; i < n; ++i) key = (key << 1) | ((x[i] >> b) & 1u);
  return key;
}

// Internal edge rows sorted along a space-filling curve through their
// midpoints (21 bits per axis over the mesh's bounding box): the Hilbert
// index, or the Morton code; ties keep the storage order. Rows close on the
// curve are close in the mesh, so the rows in flight on one XCD gather
// neighbour rows that are still in its L2; the Hilbert curve, which never
// jumps, measured 6% faster than the Morton order at 32^3 x 256.
std::vector<int32_t> curve_schedule(const Topo &T, const std::vector<int32_t> &perm, bool hilbert) {
  const int32_t ne = (int32_t)perm.size();
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int32_t v = 0; v < T.nv; ++v)
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], T.coords[3 * v + d]);
      hi[d] = std::max(hi[d], T.coords[3 * v + d]);
    }
  auto spread = [](uint64_t x) {  // 21 bits -> every third bit
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
  };
  std::vector<std::pair<uint64_t, int32_t>> key(ne);
  for (int32_t r = 0; r < ne; ++r) {
    const int32_t e = T.int_edges[perm[r]];
    const int32_t a = T.edges[2 * e], b = T.edges[2 * e + 1];
    uint64_t code = 0;
    uint32_t qx[3];
    for (int d = 0; d < 3; ++d) {
      const double m = 0.5 * (T.coords[3 * a + d] + T.coords[3 * b + d]);
      const double ext = hi[d] > lo[d] ? hi[d] - lo[d] : 1.0;
      const uint64_t qd = (uint64_t)std::min(2097151.0, std::max(0.0, (m - lo[d]) / ext * 2097151.0));
      code |= spread(qd) << d;
      qx[d] = (uint32_t)qd;
    }
    key[r] = {hilbert ? hilbert_key(qx) : code, r};
  }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> sched(ne);
  for (int32_t i = 0; i < ne; ++i) sched[i] = key[i].second;
  return sched;
}

// LDS tiles of the residual: RES_TILE consecutive rows of the visiting
// order, the sorted union of their neighbour rows and each nonzero's
// position in it. Meshes whose largest tile would not fit the LDS budget
// keep the per-wave residual (no tiles).
void residual_tiles(MeshData &md) {
  const Csr &A = md.Mp;
  const int32_t n = A.n_rows, nt = (n + RES_TILE - 1) / RES_TILE;
  md.tile_ptr.assign(nt + 1, 0);
  md.tile_cols.clear();
  md.lcol.assign(A.nnz(), 0);
  md.tile_union_max = md.tile_nnz_max = 0;
  std::vector<int32_t> cols;
  for (int32_t t = 0; t < nt; ++t) {
    cols.clear();
    int32_t nnz = 0;
    for (int32_t k = t * RES_TILE; k < std::min(n, (t + 1) * RES_TILE); ++k) {
      const int32_t r = md.sched[k];
      for (int64_t j = A.ptr[r]; j < A.ptr[r + 1]; ++j) cols.push_back(A.col[j]);
      nnz += (int32_t)(A.ptr[r + 1] - A.ptr[r]);
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    if (cols.size() > 65535) {  // lcol is 16-bit
      md.tile_ptr.clear();
      return;
    }
    for (int32_t k = t * RES_TILE; k < std::min(n, (t + 1) * RES_TILE); ++k) {
      const int32_t r = md.sched[k];
      for (int64_t j = A.ptr[r]; j < A.ptr[r + 1]; ++j)
        md.lcol[j] = (uint16_t)(std::lower_bound(cols.begin(), cols.end(), A.col[j]) - cols.begin());
    }
    md.tile_cols.insert(md.tile_cols.end(), cols.begin(), cols.end());
    md.tile_ptr[t + 1] = (int32_t)md.tile_cols.size();
    md.tile_union_max = std::max(md.tile_union_max, (int32_t)cols.size());
    md.tile_nnz_max = std::max(md.tile_nnz_max, nnz);
  }
  if (residual_tile_lds(md.tile_union_max, md.tile_nnz_max, sizeof(double)) > 65536) md.tile_ptr.clear();
}

// Row groups of the grouped residual: RES_GROUP consecutive rows of the
// visiting order, the sorted union of their neighbour rows and, per union
// entry, the mask of the group's rows coupled to it with their M and K
// entries (M and K share one pattern).
void residual_groups(MeshData &md) {
  alloc_point("residual row groups");
  const Csr &M = md.Mp, &K = md.Kp;
  const int32_t n = M.n_rows, ng = (n + RES_GROUP - 1) / RES_GROUP;
  md.gptr.assign(ng + 1, 0);
  md.gent.clear();
  md.gval.clear();
  std::vector<int32_t> cols;
  for (int32_t g = 0; g < ng; ++g) {
    const int32_t k0 = g * RES_GROUP, k1 = std::min(n, k0 + RES_GROUP);
    cols.clear();
    for (int32_t k = k0; k < k1; ++k) {
      const int32_t r = md.sched[k];
      for (int64_t j = M.ptr[r]; j < M.ptr[r + 1]; ++j) cols.push_back(M.col[j]);
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    const size_t base = md.gent.size() / 2;
    for (int32_t c : cols) {
      md.gent.push_back(c);
      md.gent.push_back(0);
    }
    md.gval.resize((base + cols.size()) * RES_GROUP * 2, 0.0);
    for (int32_t k = k0; k < k1; ++k) {
      const int32_t i = k - k0, r = md.sched[k];
      for (int64_t j = M.ptr[r]; j < M.ptr[r + 1]; ++j) {
        const size_t e = base + (size_t)(std::lower_bound(cols.begin(), cols.end(), M.col[j]) - cols.begin());
        md.gent[2 * e + 1] |= 1 << i;
        md.gval[(e * RES_GROUP + i) * 2] += M.val[j];
        md.gval[(e * RES_GROUP + i) * 2 + 1] += K.val[j];
      }
    }
    STMG_REQUIRE(base + cols.size() < (size_t)INT32_MAX, STMG_ENOMEM, "residual row groups exceed 2^31 entries");
    md.gptr[g + 1] = (int32_t)(base + cols.size());
  }
}

void setup_mesh_host(stmg_handle *h, MeshData &md) {
  SpaceLevel &S = *md.S;
  const Topo &T = S.topo;
  md.nd = nested_dissection(T, h->opt.leaf_size);
  md.sym_e = symbolic_from_tree(md.nd, edge_nodes(T, md.nd), S.M);
  if (md.index == 0)
    h->device_factor_on = !h->opt.host_only && (h->opt.device_factor > 0 ||
                                                (h->opt.device_factor < 0 && md.sym_e.nnz_L >= 1000000));
  const bool has_nodal = T.n_int_verts() > 0;
  if (has_nodal) {
    md.sym_v = symbolic_from_tree(md.nd, vertex_nodes(T, md.nd), S.Kn);
    if (h->opt.nodal > 0) {
      // no factor: K_n itself, for the Chebyshev iteration
      md.Knp = csr_permute_sym(S.Kn, md.sym_v.perm);
      double lmax = 0.0;
      for (int32_t r = 0; r < md.Knp.n_rows; ++r) {
        double sum = 0.0, diag = 0.0;
        for (int64_t k = md.Knp.ptr[r]; k < md.Knp.ptr[r + 1]; ++k) {
          sum += std::fabs(md.Knp.val[k]);
          if (md.Knp.col[k] == r) diag = md.Knp.val[k];
        }
        STMG_REQUIRE(diag > 0.0, STMG_ENUMERIC, "nodal matrix with a non-positive diagonal entry");
        lmax = std::max(lmax, sum / diag);
      }
      md.kn_lmax = lmax;
    } else if (dev_factor(h)) {
      build_front_plan(md.sym_v, S.Kn, md.fp_v);
    } else {
      md.nodal_host = std::make_unique<HostFactor<double>>();
      factor_host<double>(md.sym_v, S.Kn, S.Kn.val, *md.nodal_host);
    }
  }
  md.Mp = csr_permute_sym(S.M, md.sym_e.perm);
  md.Kp = csr_permute_sym(S.K, md.sym_e.perm);
  h->rows_hilbert = h->opt.row_schedule != 3;
  md.sched = curve_schedule(T, md.sym_e.perm, h->rows_hilbert);
  residual_tiles(md);
  residual_groups(md);
  if (dev_factor(h)) build_front_plan(md.sym_e, S.M, md.fp_e);
}

void setup_mesh_device(stmg_handle *h, MeshData &md) {
  SpaceLevel &S = *md.S;
  const Topo &T = S.topo;
  const bool has_nodal = T.n_int_verts() > 0;
  md.d_ptr = dev_upload(h, md.Mp.ptr);
  md.d_sched = dev_upload(h, md.sched);
  if (!md.tile_ptr.empty()) {
    md.d_tile_ptr = dev_upload(h, md.tile_ptr);
    md.d_tile_cols = dev_upload(h, md.tile_cols);
    md.d_lcol = dev_upload(h, md.lcol);
  }
  md.d_col = dev_upload(h, md.Mp.col);
  md.d_mval = dev_upload(h, md.Mp.val);
  md.d_kval = dev_upload(h, md.Kp.val);
  md.d_gptr = dev_upload(h, md.gptr);
  md.d_gent = dev_upload(h, md.gent);
  md.d_gval = dev_upload(h, md.gval);
  if (h->opt.precision == STMG_FP32_REFINED) {
    std::vector<float> mv(md.Mp.val.begin(), md.Mp.val.end()), kv(md.Kp.val.begin(), md.Kp.val.end());
    md.d_mval32 = dev_upload(h, mv);
    md.d_kval32 = dev_upload(h, kv);
    std::vector<float> gv(md.gval.begin(), md.gval.end());
    md.d_gval32 = dev_upload(h, gv);
  }
  const int32_t ne = T.n_int_edges(), nv = T.n_int_verts();
  // G in internal numberings
  std::vector<int32_t> head(ne, -1), tail(ne, -1);
  std::vector<int32_t> vi(nv, 0);
  if (has_nodal) vi = md.sym_v.iperm;
  for (int32_t r = 0; r < ne; ++r) {
    const int32_t asc = md.sym_e.perm[r];
    for (int64_t k = S.G.ptr[asc]; k < S.G.ptr[asc + 1]; ++k) {
      const int32_t v = vi[S.G.col[k]];
      if (S.G.val[k] > 0)
        head[r] = v;
      else
        tail[r] = v;
    }
  }
  md.d_head = dev_upload(h, head);
  md.d_tail = dev_upload(h, tail);
  std::vector<int64_t> gptr(nv + 1, 0);
  for (int32_t r = 0; r < ne; ++r) {
    if (head[r] >= 0) gptr[head[r] + 1]++;
    if (tail[r] >= 0) gptr[tail[r] + 1]++;
  }
  for (int32_t v = 0; v < nv; ++v) gptr[v + 1] += gptr[v];
  std::vector<int32_t> gedge(gptr[nv]);
  std::vector<int8_t> gsign(gptr[nv]);
  {
    std::vector<int64_t> nx(gptr.begin(), gptr.end() - 1);
    for (int32_t r = 0; r < ne; ++r) {  // ascending edge order within each vertex row
      if (head[r] >= 0) {
        gedge[nx[head[r]]] = r;
        gsign[nx[head[r]]++] = 1;
      }
      if (tail[r] >= 0) {
        gedge[nx[tail[r]]] = r;
        gsign[nx[tail[r]]++] = -1;
      }
    }
  }
  md.d_gt_ptr = dev_upload(h, gptr);
  md.d_gt_edge = dev_upload(h, gedge);
  md.d_gt_sign = dev_upload(h, gsign);
  md.d_map_level = dev_upload(h, md.sym_e.perm);
  if (md.index == 0) {
    std::vector<int32_t> abi(ne);
    for (int32_t r = 0; r < ne; ++r) abi[r] = T.int_edges[md.sym_e.perm[r]];
    md.d_map_abi = dev_upload(h, abi);
  }
  if (has_nodal && h->opt.nodal > 0) {
    const Csr &A = md.Knp;
    std::vector<double> dinv(A.n_rows, 0.0);
    for (int32_t r = 0; r < A.n_rows; ++r)
      for (int64_t k = A.ptr[r]; k < A.ptr[r + 1]; ++k)
        if (A.col[k] == r) dinv[r] = 1.0 / A.val[k];
    md.d_kn_ptr = dev_upload(h, A.ptr);
    md.d_kn_col = dev_upload(h, A.col);
    md.d_kn_val = dev_upload(h, A.val);
    md.d_kn_dinv = dev_upload(h, dinv);
    if (h->opt.precision == STMG_FP32_REFINED) {
      std::vector<float> v32(A.val.begin(), A.val.end()), d32(dinv.begin(), dinv.end());
      md.d_kn_val32 = dev_upload(h, v32);
      md.d_kn_dinv32 = dev_upload(h, d32);
    }
  } else if (has_nodal) {
    build_plan(h, md.sym_v, md.nodal);
    if (dev_factor(h)) {
      factor_into<double, float>(h, md.sym_v, md.fp_v, S.Kn.val, md.nodal, true, true,
                                 h->opt.precision == STMG_FP32_REFINED);
    } else {
      upload_factor<double, float>(h, md.sym_v, *md.nodal_host, md.nodal, true, true,
                                   h->opt.precision == STMG_FP32_REFINED);
      if (!h->opt.host_only) md.nodal_host.reset();
    }
  }
}

void setup_transfer(stmg_handle *h, MeshData &fine, MeshData &coarse) {
  // P_e (finer interior asc x coarse interior asc) -> internal numberings
  const Csr &P = coarse.S->Pe;
  Csr Pi;
  Pi.n_rows = P.n_rows;
  Pi.n_cols = P.n_cols;
  Pi.ptr.assign(P.n_rows + 1, 0);
  for (int32_t r = 0; r < P.n_rows; ++r) {
    const int32_t o = fine.sym_e.perm[r];
    Pi.ptr[r + 1] = Pi.ptr[r] + (P.ptr[o + 1] - P.ptr[o]);
  }
  for (int32_t r = 0; r < P.n_rows; ++r) {
    const int32_t o = fine.sym_e.perm[r];
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t k = P.ptr[o]; k < P.ptr[o + 1]; ++k) row.push_back({coarse.sym_e.iperm[P.col[k]], P.val[k]});
    std::sort(row.begin(), row.end());
    for (auto &e : row) {
      Pi.col.push_back(e.first);
      Pi.val.push_back(e.second);
    }
  }
  Csr Pt = csr_transpose(Pi);
  coarse.d_p_ptr = dev_upload(h, Pi.ptr);
  coarse.d_p_col = dev_upload(h, Pi.col);
  coarse.d_p_val = dev_upload(h, Pi.val);
  coarse.d_pt_ptr = dev_upload(h, Pt.ptr);
  coarse.d_pt_col = dev_upload(h, Pt.col);
  coarse.d_pt_val = dev_upload(h, Pt.val);
}

// Store P^T too when the whole hierarchy's factors fit twice in a budget
// (factor_transpose = -1), always (1) or never (0); levels with few slabs
// (solves that only stream the factor) get it under the automatic rule even
// when the budget is exceeded.
bool slab_transpose(const stmg_handle *h, const LevelData &L) {
  if (h->opt.factor_transpose == 0) return false;
  if (h->opt.factor_transpose == 1) return true;
  int64_t total = 0;
  for (const auto &l : h->levels) {
    const MeshData &md = h->meshes[h->mesh_slot[l.fmesh]];
    total += md.sym_e.panel_entries * (h->pt == 1 ? 16 : 8);
  }
  return total <= (int64_t)40 << 30 || L.N <= 16;
}

// Which slab factors each form keeps on the device: the plain form all FP64;
// the precision form FP32 on every level plus FP64 on the coarsest.
bool is_coarsest(const stmg_handle *h, const LevelData &L) { return &L == &h->levels.back(); }
bool need64(const stmg_handle *h, const LevelData &L) {
  return h->opt.precision != STMG_FP32_REFINED || is_coarsest(h, L);
}
bool need32(const stmg_handle *h, const LevelData &L) {
  return h->opt.precision == STMG_FP32_REFINED && !is_coarsest(h, L);
}

void setup_level_factor_host(stmg_handle *h, LevelData &L) {
  MeshData &md = h->meshes[h->mesh_slot[L.fmesh]];
  const SpaceLevel &S = *md.S;
  const int64_t nnz = S.M.nnz();
  if (h->pt == 1) {
    std::vector<cplx> v(nnz);
    const double s2 = std::sqrt(2.0);
    for (int64_t k = 0; k < nnz; ++k) v[k] = {2.0 * S.M.val[k] + L.tau * S.K.val[k], s2 * S.M.val[k]};
    L.slab_host_c = std::make_unique<HostFactor<cplx>>();
    factor_host<cplx>(md.sym_e, S.M, v, *L.slab_host_c);
  } else {
    std::vector<double> v(nnz);
    for (int64_t k = 0; k < nnz; ++k) v[k] = S.M.val[k] + L.tau * S.K.val[k];
    L.slab_host_r = std::make_unique<HostFactor<double>>();
    factor_host<double>(md.sym_e, S.M, v, *L.slab_host_r);
  }
}

void setup_level_factor_device(stmg_handle *h, LevelData &L) {
  MeshData &md = h->meshes[h->mesh_slot[L.fmesh]];
  const double t0 = wall_time();
  build_plan(h, md.sym_e, L.slab);
  if (verbose()) fprintf(stderr, "[stmg]   solve plan %.3fs\n", wall_time() - t0);
  if (dev_factor(h)) {
    const SpaceLevel &S = *md.S;
    const int64_t nnz = S.M.nnz();
    if (h->pt == 1) {
      std::vector<cd> v(nnz);
      const double s2 = std::sqrt(2.0);
      for (int64_t k = 0; k < nnz; ++k) v[k] = {2.0 * S.M.val[k] + L.tau * S.K.val[k], s2 * S.M.val[k]};
      L.slab.is_complex = true;
      factor_into<cd, cf>(h, md.sym_e, md.fp_e, v, L.slab, slab_transpose(h, L), need64(h, L), need32(h, L));
    } else {
      std::vector<double> v(nnz);
      for (int64_t k = 0; k < nnz; ++k) v[k] = S.M.val[k] + L.tau * S.K.val[k];
      factor_into<double, float>(h, md.sym_e, md.fp_e, v, L.slab, slab_transpose(h, L), need64(h, L),
                                 need32(h, L));
    }
    return;
  }
  if (h->pt == 1) {
    L.slab.is_complex = true;
    upload_factor<cd, cf>(h, md.sym_e, *L.slab_host_c, L.slab, slab_transpose(h, L), need64(h, L), need32(h, L));
    L.slab_host_c.reset();
  } else {
    upload_factor<double, float>(h, md.sym_e, *L.slab_host_r, L.slab, slab_transpose(h, L), need64(h, L),
                                 need32(h, L));
    L.slab_host_r.reset();
  }
}

// Diagonals of the two-grid smoother in the internal numberings: 1 / A_ii,
// A = mu M + tau K, per edge, and 1 / (mu (K_n)_vv) per vertex (complex
// pairs for DG degree 1, mu = 2 + i sqrt(2); real for degree 0, mu = 1),
// computed in FP64 and stored rounded to FP32 for the FP32 smoother.
void upload_twogrid_diagonals(stmg_handle *h, LevelData &L, const MeshData &md, bool fp32) {
  const int32_t ne = md.S->topo.n_int_edges(), nv = md.S->topo.n_int_verts();
  const bool cpx = h->pt == 1;
  const double mre = cpx ? 2.0 : 1.0, mim = cpx ? std::sqrt(2.0) : 0.0;
  auto inv = [&](double re, double im, double *out) {
    if (!cpx) {
      out[0] = 1.0 / re;
      return;
    }
    const double d = re * re + im * im;
    out[0] = re / d;
    out[1] = -im / d;
  };
  const int q = cpx ? 2 : 1;
  std::vector<double> de((size_t)ne * q), dn((size_t)std::max(nv, 1) * q, 0.0);
  for (int32_t r = 0; r < ne; ++r) {
    double m = 0.0, k = 0.0;
    for (int64_t j = md.Mp.ptr[r]; j < md.Mp.ptr[r + 1]; ++j)
      if (md.Mp.col[j] == r) {
        m = md.Mp.val[j];
        k = md.Kp.val[j];
      }
    STMG_REQUIRE(m > 0.0, STMG_ENUMERIC, "mass matrix with a non-positive diagonal entry");
    inv(mre * m + L.tau * k, mim * m, &de[(size_t)r * q]);
  }
  const Csr &Kn = md.S->Kn;
  for (int32_t r = 0; r < nv; ++r) {
    const int32_t a = md.sym_v.perm[r];  // internal vertex r -> ascending interior index
    double kd = 0.0;
    for (int64_t j = Kn.ptr[a]; j < Kn.ptr[a + 1]; ++j)
      if (Kn.col[j] == a) kd = Kn.val[j];
    STMG_REQUIRE(kd > 0.0, STMG_ENUMERIC, "nodal matrix with a non-positive diagonal entry");
    inv(mre * kd, mim * kd, &dn[(size_t)r * q]);
  }
  if (fp32) {  // the FP32 smoother's copies
    L.tg_dinv32 = dev_upload(h, std::vector<float>(de.begin(), de.end()));
    L.tg_dn32 = dev_upload(h, std::vector<float>(dn.begin(), dn.end()));
  } else {
    L.tg_dinv = dev_upload(h, de);
    L.tg_dn = dev_upload(h, dn);
  }
}

void alloc_level_vectors(stmg_handle *h, LevelData &L, bool first) {
  MeshData &md = h->meshes[h->mesh_slot[L.mesh]];
  const int64_t ne = md.S->topo.n_int_edges(), nv = md.S->topo.n_int_verts();
  const int64_t W = (int64_t)L.N * h->q;
  const bool prec = h->opt.precision == STMG_FP32_REFINED;
  const bool last = is_coarsest(h, L);
  // FP64: every level in the plain form; in the precision form the outer
  // iterate, right-hand side and residual on level 0 and the coarsest solve
  if (!prec || first || last) {
    L.x = dev_alloc<double>(h, ne * W);
    L.b = dev_alloc<double>(h, ne * W);
    L.w = dev_alloc<double>(h, ne * W);
  }
  if (!prec || last) {
    L.z = dev_alloc<double>(h, ne * W);
    L.u = dev_alloc<double>(h, std::max<int64_t>(1, L.slab.u_rows * W));
  }
  const bool cheb = h->opt.nodal > 0;
  if (!prec && nv > 0) {
    L.g = dev_alloc<double>(h, nv * W);
    L.zn = dev_alloc<double>(h, nv * W);
    L.un = dev_alloc<double>(h, std::max<int64_t>(1, (cheb ? nv : md.nodal.u_rows) * W));
    if (cheb) L.yn = dev_alloc<double>(h, nv * W);
  }
  if (L.twogrid) {  // in the precision form the FP32 smoother's buffers only
    const MeshData &mf = h->meshes[h->mesh_slot[L.fmesh]];
    const int64_t nc = (int64_t)mf.S->topo.n_int_edges() * W;
    if (prec) {
      if (h->opt.slab > 1) L.tg_r32 = dev_alloc<float>(h, ne * W);
      L.tg_a32 = dev_alloc<float>(h, ne * W);
      L.tg_b32 = dev_alloc<float>(h, ne * W);
      L.tg_t32 = dev_alloc<float>(h, ne * W);
      L.tg_c32 = dev_alloc<float>(h, nc);
    } else {
      if (h->opt.slab > 1) L.tg_r = dev_alloc<double>(h, ne * W);
      L.tg_a = dev_alloc<double>(h, ne * W);
      L.tg_b = dev_alloc<double>(h, ne * W);
      L.tg_t = dev_alloc<double>(h, ne * W);
      L.tg_c = dev_alloc<double>(h, nc);
    }
    upload_twogrid_diagonals(h, L, md, prec);
  }
  if (prec && first && last) {
    L.xe = dev_alloc<double>(h, ne * W);
    L.be = dev_alloc<double>(h, ne * W);
  }
  if (prec) {
    L.x32 = dev_alloc<float>(h, ne * W);
    L.b32 = dev_alloc<float>(h, ne * W);
    L.w32 = dev_alloc<float>(h, ne * W);
    L.z32 = dev_alloc<float>(h, ne * W);
    L.u32 = dev_alloc<float>(h, std::max<int64_t>(1, L.slab.u_rows * W));
    if (nv > 0) {
      L.g32 = dev_alloc<float>(h, nv * W);
      L.zn32 = dev_alloc<float>(h, nv * W);
      L.un32 = dev_alloc<float>(h, std::max<int64_t>(1, (cheb ? nv : md.nodal.u_rows) * W));
      if (cheb) L.yn32 = dev_alloc<float>(h, nv * W);
    }
  }
}

// --------------------------------------------------------------- operators
// Buffer and factor selection by precision: R = double is the plain FP64
// form; R = float the smoother of the precision form (FP32 vectors, matrix
// values and factors), whose coarsest solve runs in FP64.
template <typename R>
struct Bufs;
template <>
struct Bufs<double> {
  static double *x(LevelData &L) { return L.x; }
  static double *b(LevelData &L) { return L.b; }
  static double *w(LevelData &L) { return L.w; }
  static double *z(LevelData &L) { return L.z; }
  static double *u(LevelData &L) { return L.u; }
  static double *g(LevelData &L) { return L.g; }
  static double *zn(LevelData &L) { return L.zn; }
  static double *un(LevelData &L) { return L.un; }
  static double *yn(LevelData &L) { return L.yn; }
  static const double *knval(MeshData &m) { return m.d_kn_val; }
  static const double *kndinv(MeshData &m) { return m.d_kn_dinv; }
  static const double *mval(MeshData &m) { return m.d_mval; }
  static const double *kval(MeshData &m) { return m.d_kval; }
  static const double *gval(MeshData &m) { return m.d_gval; }
  static const FactorDev &fac(DevFactor &d) { return d.f; }
  static double *tg_dinv(LevelData &L) { return L.tg_dinv; }
  static double *tg_dn(LevelData &L) { return L.tg_dn; }
  static double *tg_r(LevelData &L) { return L.tg_r; }
  static double *tg_a(LevelData &L) { return L.tg_a; }
  static double *tg_b(LevelData &L) { return L.tg_b; }
  static double *tg_t(LevelData &L) { return L.tg_t; }
  static double *tg_c(LevelData &L) { return L.tg_c; }
  using C = cd;
};
template <>
struct Bufs<float> {
  static float *x(LevelData &L) { return L.x32; }
  static float *b(LevelData &L) { return L.b32; }
  static float *w(LevelData &L) { return L.w32; }
  static float *z(LevelData &L) { return L.z32; }
  static float *u(LevelData &L) { return L.u32; }
  static float *g(LevelData &L) { return L.g32; }
  static float *zn(LevelData &L) { return L.zn32; }
  static float *un(LevelData &L) { return L.un32; }
  static float *yn(LevelData &L) { return L.yn32; }
  static const float *knval(MeshData &m) { return m.d_kn_val32; }
  static const float *kndinv(MeshData &m) { return m.d_kn_dinv32; }
  static const float *mval(MeshData &m) { return m.d_mval32; }
  static const float *kval(MeshData &m) { return m.d_kval32; }
  static const float *gval(MeshData &m) { return m.d_gval32; }
  static const FactorDev &fac(DevFactor &d) { return d.f32; }
  static float *tg_dinv(LevelData &L) { return L.tg_dinv32; }
  static float *tg_dn(LevelData &L) { return L.tg_dn32; }
  static float *tg_r(LevelData &L) { return L.tg_r32; }
  static float *tg_a(LevelData &L) { return L.tg_a32; }
  static float *tg_b(LevelData &L) { return L.tg_b32; }
  static float *tg_t(LevelData &L) { return L.tg_t32; }
  static float *tg_c(LevelData &L) { return L.tg_c32; }
  using C = cf;
};

// Name of each smoother option as section 4 writes it (a product of S and A
// steps, applied right to left when pre-smoothing).
const char *smoother_sequence(int32_t v) {
  switch (v) {
    case STMG_SMOOTH_SAS: return "SAS";
    case STMG_SMOOTH_S_ONLY: return "SS";
    case STMG_SMOOTH_SA: return "SA";
    case STMG_SMOOTH_AS: return "AS";
    case STMG_SMOOTH_SSA: return "SSA";
    case STMG_SMOOTH_ASS: return "ASS";
    case STMG_SMOOTH_SSAS: return "SSAS";
    case STMG_SMOOTH_SSASS: return "SSASS";
    default: return nullptr;
  }
}

template <typename R>
struct OpsT {
  stmg_handle *h;
  hipStream_t s;
  using B = Bufs<R>;
  using CX = typename B::C;

  MeshData &mesh(int l) { return h->meshes[h->mesh_slot[h->levels[l].mesh]]; }
  int32_t ne(int l) { return mesh(l).S->topo.n_int_edges(); }
  int32_t nv(int l) { return mesh(l).S->topo.n_int_verts(); }
  int32_t W(int l) { return h->levels[l].N * h->q; }
  bool coarsest(int l) { return l + 1 == (int)h->levels.size(); }

  // returns the number of norm partials written (when partial is set)
  int residual(int l, const R *x, const R *b, R *out, int mode, double *partial) {
    MeshData &md = mesh(l);
    ResidualArgsT<R> a;
    a.n_rows = ne(l);
    a.N = h->levels[l].N;
    a.q = h->q;
    a.ptr = md.d_ptr;
    a.col = md.d_col;
    a.mval = B::mval(md);
    a.kval = B::kval(md);
    a.tau = h->levels[l].tau;
    a.x = x;
    a.b = b;
    a.out = out;
    a.partial = partial;
    a.mode = mode;
    a.nnz = md.Mp.nnz();
    a.prof = h->prof_state.on ? &h->prof : nullptr;
    a.chunk = h->opt.stream_chunk;
    a.halo = h->d_halo;
    a.sched = h->opt.row_schedule != 1 ? md.d_sched : nullptr;
    if (h->opt.row_schedule == 0 || h->opt.row_schedule == 3) {
      a.gptr = md.d_gptr;
      a.gent = md.d_gent;
      a.gval = B::gval(md);
    }
    if (a.sched && md.d_tile_ptr) {
      a.tile_ptr = md.d_tile_ptr;
      a.tile_cols = md.d_tile_cols;
      a.lcol = md.d_lcol;
      a.tile_union_max = md.tile_union_max;
      a.tile_nnz_max = md.tile_nnz_max;
    }
    return launch_residual(a, s);
  }

  // Streaming kernels under the per-launch profiler (algorithmic bytes:
  // each operand read once, each result written once).
  template <typename Fn>
  void timed(const char *base, double bytes, Fn &&fn) {
    if (!h->prof_state.on) {
      fn();
      return;
    }
    char name[64];
    snprintf(name, sizeof name, "%s<%s>", base, sizeof(R) == 8 ? "double" : "float");
    h->prof.begin(s);
    fn();
    h->prof.end(s, name, 0.0, bytes);
  }

  // w <- A_l^{-1} w in place (slab right-hand-side layout); inexactly on
  // levels with two-grid slab solves
  void slab_solve(int l, R *w) {
    LevelData &L = h->levels[l];
    if (L.twogrid) {
      if (L.slab.is_complex)
        slab_solve_twogrid<CX>(l, w);
      else
        slab_solve_twogrid<R>(l, w);
      return;
    }
    const int32_t nc = L.N;
    const FactorDev &F = B::fac(L.slab);
    if (L.slab.is_complex) {
      solve_forward<CX>(F, L.slab.plan, nc, (CX *)w, (CX *)B::z(L), (CX *)B::u(L), s);
      solve_backward<CX>(F, L.slab.plan, nc, (CX *)w, (CX *)B::z(L), s);
    } else {
      solve_forward<R>(F, L.slab.plan, nc, w, B::z(L), B::u(L), s);
      solve_backward<R>(F, L.slab.plan, nc, w, B::z(L), s);
    }
  }

  // Two-grid slab solve (option slab = k): w <- k steps of Richardson
  // iteration from zero for A z = w, z <- z + B (w - A z), A = mu M + tau K
  // on the level's mesh (T = cd: mu = 2 + i sqrt(2); T = double: mu = 1),
  // one scalar per slab and row. B is one two-grid cycle (section 5's
  // inexact spatial solves): two sweeps of [damped edge Jacobi, omega 1/2;
  // Jacobi on the gradients with diag(mu K_n)], the exact solve of
  // mu M_c + tau K_c on the next coarser mesh between the transfers P^T and
  // P, then the two sweeps with their steps reversed.
  template <typename T>
  void slab_solve_twogrid(int l, R *w_) {
    LevelData &L = h->levels[l];
    MeshData &md = mesh(l);
    MeshData &mc = h->meshes[h->mesh_slot[L.fmesh]];
    const int32_t n = ne(l), nvl = nv(l), N = L.N, ncl = mc.S->topo.n_int_edges(), wl = W(l);
    const double tau = L.tau, om = 0.5, sz = sizeof(R);
    T mu;
    if constexpr (std::is_same<T, CX>::value)
      mu = CX{(R)2.0, (R)std::sqrt(2.0)};
    else
      mu = (R)1.0;
    const T *dinv = (const T *)B::tg_dinv(L), *dn = (const T *)B::tg_dn(L);
    T *w = (T *)w_, *t = (T *)B::tg_t(L), *c = (T *)B::tg_c(L);
    R *g = B::g(L);
    const double vec = sz * wl * n, pat = (double)md.Mp.nnz() * (4 + 2 * sz) + 8.0 * n;
    // out = r - A z (mode 0); out = z + om dinv (r - A z) (mode 1, out != z,
    // out may be r); out = om dinv r (mode 2)
    auto apply = [&](const T *r, const T *z, T *out, int mode) {
      timed("k_tg_apply", mode == 2 ? 2.0 * vec : 3.0 * vec + pat + (mode == 1 ? sz * wl * n / N : 0.0), [&] {
        launch_tg_apply<T>(n, N, md.d_sched, md.d_ptr, md.d_col, B::mval(md), B::kval(md), mu, tau, dinv, om, r, z,
                           out, mode, s);
      });
    };
    auto nodal = [&](const T *r, T *z) {
      if (nvl == 0) return;
      apply(r, z, t, 0);
      timed("k_gradT", sz * wl * ((double)n + nvl), [&] {
        launch_gradT<R>(nvl, wl, md.d_gt_ptr, md.d_gt_edge, md.d_gt_sign, (const R *)t, g, s);
      });
      timed("k_scale_slabs", 2.0 * sz * wl * nvl, [&] { launch_scale_slabs<T>(nvl, N, dn, (T *)g, s); });
      timed("k_grad_add", sz * wl * ((double)nvl + 2.0 * n),
            [&] { launch_grad_add<R>(n, wl, md.d_head, md.d_tail, g, (R *)z, s); });
    };
    auto coarse = [&](const T *r, T *z) {
      apply(r, z, t, 0);
      timed("k_csr_slabs", sz * wl * ((double)n + ncl),
            [&] { launch_csr_slabs<T>(ncl, N, mc.d_pt_ptr, mc.d_pt_col, mc.d_pt_val, t, c, 0, s); });
      // t is free again: the coarse solve's workspace
      const FactorDev &F = B::fac(L.slab);
      solve_forward<T>(F, L.slab.plan, N, c, t, (T *)B::u(L), s);
      solve_backward<T>(F, L.slab.plan, N, c, t, s);
      timed("k_csr_slabs", sz * wl * ((double)ncl + 2.0 * n),
            [&] { launch_csr_slabs<T>(n, N, mc.d_p_ptr, mc.d_p_col, mc.d_p_val, c, z, 1, s); });
    };
    // out <- B r with iterates in a and b; out != a (out may be b or r)
    auto precondition = [&](const T *r, T *a, T *b, T *out) {
      apply(r, nullptr, a, 2);
      nodal(r, a);
      apply(r, a, b, 1);
      nodal(r, b);
      coarse(r, b);
      nodal(r, b);
      apply(r, b, a, 1);
      nodal(r, a);
      apply(r, a, out, 1);
    };
    T *a = (T *)B::tg_a(L), *b = (T *)B::tg_b(L), *z = (T *)B::z(L), *rho = (T *)B::tg_r(L);
    const int k = h->opt.slab;
    const int64_t nd = (int64_t)n * wl;
    if (k == 1) {
      precondition(w, a, b, w);
      return;
    }
    precondition(w, a, b, z);
    for (int j = 2; j <= k; ++j) {
      apply(w, z, rho, 0);
      if (j < k) {
        precondition(rho, a, b, b);
        timed("k_tg_axpy", 3.0 * sz * nd, [&] { launch_tg_axpy<R>(nd, (const R *)b, (R *)z, s); });
      } else {  // the last step writes z + B rho over w
        precondition(rho, a, b, w);
        timed("k_tg_axpy", 3.0 * sz * nd, [&] { launch_tg_axpy<R>(nd, (const R *)z, (R *)w, s); });
      }
    }
  }

  void smooth_S(int l, R *x, const R *b) {
    LevelData &L = h->levels[l];
    residual(l, x, b, B::w(L), RES_OUT_SLABRHS, nullptr);
    slab_solve(l, B::w(L));
    timed("k_slab_update", 3.0 * sizeof(R) * ne(l) * W(l),
          [&] { launch_slab_update<R>(ne(l), L.N, h->q, h->opt.omega, B::w(L), x, 0, s); });
  }

  void nodal_A(int l, R *x, const R *b) {
    LevelData &L = h->levels[l];
    MeshData &md = mesh(l);
    if (nv(l) == 0) return;
    const int32_t w = W(l);
    residual(l, x, b, B::w(L), RES_OUT_R, nullptr);
    const double sz = sizeof(R);
    timed("k_gradT", sz * w * ((double)ne(l) + nv(l)),
          [&] { launch_gradT<R>(nv(l), w, md.d_gt_ptr, md.d_gt_edge, md.d_gt_sign, B::w(L), B::g(L), s); });
    R *y = nodal_solve(l);
    timed("k_time_scan", 2.0 * sz * w * nv(l), [&] { launch_time_scan<R>(nv(l), L.N, h->q, y, s); });
    timed("k_grad_add", sz * w * ((double)nv(l) + 2.0 * ne(l)),
          [&] { launch_grad_add<R>(ne(l), w, md.d_head, md.d_tail, y, x, s); });
  }

  // y = K_n^{-1} g for every column of g (level l's g buffer): exactly with
  // the factor, in place; or (option nodal = k > 0) k steps of the
  // Jacobi-preconditioned Chebyshev iteration on [lmax / 30, lmax], lmax the
  // Gershgorin bound of D^{-1} K_n (section 5's inexact spatial solves).
  // Returns the buffer that holds y.
  R *nodal_solve(int l) {
    LevelData &L = h->levels[l];
    MeshData &md = mesh(l);
    const int32_t w = W(l);
    if (h->opt.nodal <= 0) {
      const FactorDev &F = B::fac(md.nodal);
      solve_forward<R>(F, md.nodal.plan, w, B::g(L), B::zn(L), B::un(L), s);
      solve_backward<R>(F, md.nodal.plan, w, B::g(L), B::zn(L), s);
      return B::g(L);
    }
    const double lmax = md.kn_lmax, lmin = lmax / 30.0;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
    double rho = 1.0 / sigma;
    R *ya = B::un(L), *yb = B::yn(L), *d = B::zn(L);
    const double bytes = sizeof(R) * (double)w * nv(l);
    timed("k_cheb_step", 3.0 * bytes, [&] {
      launch_cheb_step<R>(nv(l), w, md.d_kn_ptr, md.d_kn_col, B::knval(md), B::kndinv(md), B::g(L), nullptr, d,
                          ya, 0.0, 1.0 / theta, s);
    });
    for (int i = 1; i < h->opt.nodal; ++i) {
      const double rho_new = 1.0 / (2.0 * sigma - rho);
      timed("k_cheb_step", 5.0 * bytes, [&] {
        launch_cheb_step<R>(nv(l), w, md.d_kn_ptr, md.d_kn_col, B::knval(md), B::kndinv(md), B::g(L), ya, d, yb,
                            rho_new * rho, 2.0 * rho_new / delta, s);
      });
      std::swap(ya, yb);
      rho = rho_new;
    }
    return ya;
  }

  // The handle's smoother of S and A steps (section 4). Its name reads like
  // a product of matrices, right to left (SA = A, then S), before the
  // coarse-grid correction; after it the same steps run in reversed order.
  void hybrid(int l, R *x, const R *b, bool pre) {
    const char *seq = smoother_sequence(h->opt.smoother);
    const int n = (int)strlen(seq);
    for (int i = 0; i < n; ++i) {
      if (seq[pre ? n - 1 - i : i] == 'S')
        smooth_S(l, x, b);
      else
        nodal_A(l, x, b);
    }
  }

  void exact(int l, R *x, const R *b);

  void restrict_to(int l, const R *rf, R *rc) {
    LevelData &C = h->levels[l + 1];
    const double bytes = sizeof(R) * ((double)ne(l) * W(l) + (double)ne(l + 1) * W(l + 1));
    timed("k_restrict", bytes, [&] {
      if (C.mesh != h->levels[l].mesh) {
        MeshData &mc = mesh(l + 1);
        launch_restrict<R>(ne(l + 1), C.N, h->q, mc.d_pt_ptr, mc.d_pt_col, mc.d_pt_val, rf, rc, s);
      } else {
        launch_restrict<R>(ne(l + 1), C.N, h->q, nullptr, nullptr, nullptr, rf, rc, s);
      }
    });
  }

  void prolong_add(int l, const R *ec, R *xf) {
    // from level l+1 to level l
    LevelData &C = h->levels[l + 1];
    const double bytes = sizeof(R) * (2.0 * ne(l) * W(l) + (double)ne(l + 1) * W(l + 1));
    timed("k_prolong_add", bytes, [&] {
      if (C.mesh != h->levels[l].mesh) {
        MeshData &mc = mesh(l + 1);
        launch_prolong_add<R>(ne(l), C.N, h->q, mc.d_p_ptr, mc.d_p_col, mc.d_p_val, ec, xf, s);
      } else {
        launch_prolong_add<R>(ne(l), C.N, h->q, nullptr, nullptr, nullptr, ec, xf, s);
      }
    });
  }

  void vcycle(int l, R *x, const R *b) {
    LevelData &L = h->levels[l];
    if (L.N == 1) {
      exact(l, x, b);
      return;
    }
    hybrid(l, x, b, true);
    residual(l, x, b, B::w(L), RES_OUT_R, nullptr);
    LevelData &C = h->levels[l + 1];
    restrict_to(l, B::w(L), B::b(C));
    launch_fill<R>(B::x(C), (int64_t)ne(l + 1) * W(l + 1), 0.0, s);
    vcycle(l + 1, B::x(C), B::b(C));
    prolong_add(l, B::x(C), x);
    hybrid(l, x, b, false);
  }

  // ||b - L x||^2 into dst (device), FP64 accumulation
  void residual_norm2(int l, const R *x, const R *b, R *out, double *dst) {
    const int nb = residual(l, x, b, out, RES_OUT_R, h->d_partial);
    launch_sum(h->d_partial, nb, dst, s);
  }
};

// Exact solve with the slab factor on a one-slab level (FP64 factor).
template <>
void OpsT<double>::exact(int l, double *x, const double *b) {
  LevelData &L = h->levels[l];
  launch_slab_rhs<double>(ne(l), L.N, h->q, b, L.w, s);
  slab_solve(l, L.w);
  launch_slab_update<double>(ne(l), L.N, h->q, 1.0, L.w, x, 1, s);
}

// The precision form keeps the coarsest solve in FP64: widen b, solve with
// the FP64 factor, narrow x. When the coarsest level is level 0 (one slab),
// its x and b hold the outer FP64 iterate and right-hand side, so the solve
// works in buffers of its own.
template <>
void OpsT<float>::exact(int l, float *x, const float *b) {
  LevelData &L = h->levels[l];
  const int64_t n = (int64_t)ne(l) * W(l);
  double *xd = L.xe ? L.xe : L.x, *bd = L.be ? L.be : L.b;
  launch_to_double(n, b, bd, s);
  OpsT<double>{h, s}.exact(l, xd, bd);
  launch_to_float(n, xd, x, s);
}

using Ops = OpsT<double>;

// One iteration of the precision form on level 0: e = V32(r) from e = 0,
// x += e in FP64, then the FP64 residual r = b - L x and its squared norm.
void refine_iteration(stmg_handle *h, double *dst_norm2) {
  OpsT<float> o32{h, h->stream};
  Ops o64{h, h->stream};
  LevelData &L = h->levels[0];
  const int64_t n = (int64_t)o64.ne(0) * o64.W(0);
  launch_to_float(n, L.w, L.b32, h->stream);
  launch_fill<float>(L.x32, n, 0.0, h->stream);
  o32.vcycle(0, L.x32, L.b32);
  launch_add_float(n, L.x32, L.x, h->stream);
  o64.residual_norm2(0, L.x, L.b, L.w, dst_norm2);
}

// One solver iteration on level 0 (either form); ||b - L x||^2 into dst.
void solver_iteration(stmg_handle *h, double *dst_norm2) {
  if (h->opt.precision == STMG_FP32_REFINED) {
    refine_iteration(h, dst_norm2);
  } else {
    Ops op{h, h->stream};
    LevelData &L = h->levels[0];
    op.vcycle(0, L.x, L.b);
    op.residual_norm2(0, L.x, L.b, L.w, dst_norm2);
  }
}

// ---------------------------------------------------------- batched cycles
// One iteration for several handles at once. The members share N_t, p_t,
// the precision form and the smoother sequence, so their V-cycles take the
// same sequence of level steps; the streaming steps (residual, Jacobi
// update, G^T, time scan, G-add, transfers) run per member on the shared
// stream, the slab and nodal solves of each step run merged over the
// members (one launch per tree height and tile shape). Each member's values
// are computed by the same instructions in the same order as in its own
// iteration, so batched and separate iterations agree bitwise.
template <typename R>
struct GroupOps {
  std::vector<OpsT<R>> ops;
  hipStream_t s;
  using B = Bufs<R>;
  using CX = typename B::C;

  static LevelData &lev(OpsT<R> &o, int l) { return o.h->levels[l]; }

  // exact slab solves merged over the members; two-grid ones member by member
  void slab_solves(int l) {
    for (auto &o : ops)
      if (lev(o, l).twogrid) o.slab_solve(l, B::w(lev(o, l)));
    if (lev(ops[0], l).slab.is_complex) {
      std::vector<SolveMember<CX>> m;
      for (auto &o : ops) {
        LevelData &L = lev(o, l);
        if (!L.twogrid)
          m.push_back({&B::fac(L.slab), &L.slab.plan, L.N, (CX *)B::w(L), (CX *)B::z(L), (CX *)B::u(L)});
      }
      if (!m.empty()) {
        solve_forward_group<CX>(m.data(), (int)m.size(), s);
        solve_backward_group<CX>(m.data(), (int)m.size(), s);
      }
    } else {
      std::vector<SolveMember<R>> m;
      for (auto &o : ops) {
        LevelData &L = lev(o, l);
        if (!L.twogrid) m.push_back({&B::fac(L.slab), &L.slab.plan, L.N, B::w(L), B::z(L), B::u(L)});
      }
      if (!m.empty()) {
        solve_forward_group<R>(m.data(), (int)m.size(), s);
        solve_backward_group<R>(m.data(), (int)m.size(), s);
      }
    }
  }

  void smooth_S(int l) {
    for (auto &o : ops) {
      LevelData &L = lev(o, l);
      o.residual(l, B::x(L), B::b(L), B::w(L), RES_OUT_SLABRHS, nullptr);
    }
    slab_solves(l);
    for (auto &o : ops) {
      LevelData &L = lev(o, l);
      launch_slab_update<R>(o.ne(l), L.N, o.h->q, o.h->opt.omega, B::w(L), B::x(L), 0, s);
    }
  }

  void nodal_A(int l) {
    if (ops[0].h->opt.nodal > 0) {  // inexact nodal solves: per member
      for (auto &o : ops) o.nodal_A(l, B::x(lev(o, l)), B::b(lev(o, l)));
      return;
    }
    std::vector<SolveMember<R>> m;
    for (auto &o : ops) {
      if (o.nv(l) == 0) continue;
      LevelData &L = lev(o, l);
      MeshData &md = o.mesh(l);
      o.residual(l, B::x(L), B::b(L), B::w(L), RES_OUT_R, nullptr);
      launch_gradT<R>(o.nv(l), o.W(l), md.d_gt_ptr, md.d_gt_edge, md.d_gt_sign, B::w(L), B::g(L), s);
      m.push_back({&B::fac(md.nodal), &md.nodal.plan, o.W(l), B::g(L), B::zn(L), B::un(L)});
    }
    solve_forward_group<R>(m.data(), (int)m.size(), s);
    solve_backward_group<R>(m.data(), (int)m.size(), s);
    for (auto &o : ops) {
      if (o.nv(l) == 0) continue;
      LevelData &L = lev(o, l);
      MeshData &md = o.mesh(l);
      launch_time_scan<R>(o.nv(l), L.N, o.h->q, B::g(L), s);
      launch_grad_add<R>(o.ne(l), o.W(l), md.d_head, md.d_tail, B::g(L), B::x(L), s);
    }
  }

  void hybrid(int l, bool pre) {
    const char *seq = smoother_sequence(ops[0].h->opt.smoother);
    const int n = (int)strlen(seq);
    for (int i = 0; i < n; ++i) {
      if (seq[pre ? n - 1 - i : i] == 'S')
        smooth_S(l);
      else
        nodal_A(l);
    }
  }

  void vcycle(int l) {
    if (lev(ops[0], l).N == 1) {
      for (auto &o : ops) o.exact(l, B::x(lev(o, l)), B::b(lev(o, l)));
      return;
    }
    hybrid(l, true);
    for (auto &o : ops) {
      LevelData &L = lev(o, l), &C = lev(o, l + 1);
      o.residual(l, B::x(L), B::b(L), B::w(L), RES_OUT_R, nullptr);
      o.restrict_to(l, B::w(L), B::b(C));
      launch_fill<R>(B::x(C), (int64_t)o.ne(l + 1) * o.W(l + 1), 0.0, s);
    }
    vcycle(l + 1);
    for (auto &o : ops) o.prolong_add(l, B::x(lev(o, l + 1)), B::x(lev(o, l)));
    hybrid(l, false);
  }
};

// Handles that may share a batched iteration: the same N_t, DG degree,
// precision form and smoother sequence (so the same steps in the same order).
bool same_cycle_shape(const stmg_handle *a, const stmg_handle *b) {
  return a->Nt == b->Nt && a->pt == b->pt && a->opt.precision == b->opt.precision &&
         a->opt.smoother == b->opt.smoother && a->opt.nodal == b->opt.nodal && a->opt.slab == b->opt.slab &&
         a->levels.size() == b->levels.size();
}

// One iteration of every member on stream s; ||b - L x||^2 into each
// member's d_scalar[slot].
void group_iteration(const std::vector<stmg_handle *> &hs, hipStream_t s, int slot) {
  if (hs[0]->opt.precision == STMG_FP32_REFINED) {
    GroupOps<float> g;
    g.s = s;
    for (auto *h : hs) {
      LevelData &L = h->levels[0];
      OpsT<float> o{h, s};
      const int64_t n = (int64_t)o.ne(0) * o.W(0);
      launch_to_float(n, L.w, L.b32, s);
      launch_fill<float>(L.x32, n, 0.0, s);
      g.ops.push_back(o);
    }
    g.vcycle(0);
    for (auto *h : hs) {
      LevelData &L = h->levels[0];
      Ops o64{h, s};
      launch_add_float((int64_t)o64.ne(0) * o64.W(0), L.x32, L.x, s);
      o64.residual_norm2(0, L.x, L.b, L.w, h->d_scalar + slot);
    }
  } else {
    GroupOps<double> g;
    g.s = s;
    for (auto *h : hs) g.ops.push_back(Ops{h, s});
    g.vcycle(0);
    for (auto *h : hs) {
      LevelData &L = h->levels[0];
      Ops{h, s}.residual_norm2(0, L.x, L.b, L.w, h->d_scalar + slot);
    }
  }
}

void check_launch() { hip_check(hipGetLastError(), "kernel launch"); }

// ------------------------------------------------------- graph replay
// The launches of one iteration are the same in every cycle (same buffers,
// shapes and arguments), so they are captured once on a private stream into
// a HIP graph and replayed on the handle's stream: the launch sequence goes
// to the device in one call, and the iterate is bitwise that of the eager
// launches. The iteration holds no memory set or copy nodes; its norm goes
// to d_scalar[GRAPH_NORM_SLOT].
void drop_graph(stmg_handle *h) {
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  h->graph_exec = nullptr;
}

bool use_graph(const stmg_handle *h) { return h->opt.graph != 0 && !h->prof_state.on; }

void capture_iteration(stmg_handle *h) {
  if (h->graph_exec) return;
  if (!h->graph_stream) hip_check(hipStreamCreateWithFlags(&h->graph_stream, hipStreamNonBlocking), "hipStreamCreate");
  hipStream_t user = h->stream;
  h->stream = h->graph_stream;
  hipGraph_t g = nullptr;
  hip_check(hipStreamBeginCapture(h->graph_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  try {
    solver_iteration(h, h->d_scalar + GRAPH_NORM_SLOT);
  } catch (...) {
    (void)hipStreamEndCapture(h->graph_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    h->stream = user;
    throw;
  }
  h->stream = user;
  hip_check(hipStreamEndCapture(h->graph_stream, &g), "hipStreamEndCapture");
  const hipError_t e = hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hip_check(e, "hipGraphInstantiate");
}

// One iteration on the handle's stream, replayed from the graph or launched
// eagerly; the squared residual norm ends in dst (device).
void run_iteration(stmg_handle *h, double *dst) {
  if (!use_graph(h)) {
    solver_iteration(h, dst);
    return;
  }
  capture_iteration(h);
  hip_check(hipGraphLaunch(h->graph_exec, h->stream), "hipGraphLaunch");
  if (dst != h->d_scalar + GRAPH_NORM_SLOT)
    hip_check(hipMemcpyAsync(dst, h->d_scalar + GRAPH_NORM_SLOT, sizeof(double), hipMemcpyDeviceToDevice, h->stream),
              "copy");
}

void set_profiler(stmg_handle *h, bool on) {
  Profiler *p = on ? &h->prof : nullptr;
  for (auto &L : h->levels) L.slab.plan.prof = p;
  for (auto &m : h->meshes) m.nodal.plan.prof = p;
}

// Setup progress on stderr when STMG_VERBOSE is set (long factorisations).

void require_device(const stmg_handle *h) {
  STMG_REQUIRE(h, STMG_EINVAL, "null handle");
  STMG_REQUIRE(!h->opt.host_only, STMG_ENOSYS, "handle was built with host_only");
}

double *tmp_buf(stmg_handle *h, int i) {
  if (!h->d_tmp[i]) {
    const LevelData &L = h->levels[0];
    const MeshData &md = h->meshes[h->mesh_slot[L.mesh]];
    h->d_tmp[i] = dev_alloc<double>(h, (size_t)md.S->topo.n_int_edges() * L.N * h->q);
  }
  return h->d_tmp[i];
}

float *tmp_buf32(stmg_handle *h, int i) {
  if (!h->f_tmp[i]) {
    const LevelData &L = h->levels[0];
    const MeshData &md = h->meshes[h->mesh_slot[L.mesh]];
    h->f_tmp[i] = dev_alloc<float>(h, (size_t)md.S->topo.n_int_edges() * L.N * h->q);
  }
  return h->f_tmp[i];
}

// One level operation on internal-layout buffers t0 (x or input), t1 (b),
// result in t2.
template <typename R>
void apply_op(stmg_handle *h, int level, int op_code, R *t0, R *t1, R *t2) {
  OpsT<R> op{h, h->stream};
  hipStream_t s = h->stream;
  LevelData &L = h->levels[level];
  const int32_t ne = op.ne(level);
  const size_t bytes = (size_t)ne * op.W(level) * sizeof(R);
  switch (op_code) {
    case STMG_OP_RESIDUAL:
      op.residual(level, t0, t1, t2, RES_OUT_R, nullptr);
      break;
    case STMG_OP_SMOOTH_S:
    case STMG_OP_NODAL_A:
    case STMG_OP_SAS:
    case STMG_OP_VCYCLE:
      hip_check(hipMemcpyAsync(t2, t0, bytes, hipMemcpyDeviceToDevice, s), "copy");
      if (op_code == STMG_OP_SMOOTH_S) op.smooth_S(level, t2, t1);
      if (op_code == STMG_OP_NODAL_A) op.nodal_A(level, t2, t1);
      if (op_code == STMG_OP_SAS) op.hybrid(level, t2, t1, true);
      if (op_code == STMG_OP_VCYCLE) op.vcycle(level, t2, t1);
      break;
    case STMG_OP_SLAB_SOLVE:
      launch_slab_rhs<R>(ne, L.N, h->q, t0, Bufs<R>::w(L), s);
      op.slab_solve(level, Bufs<R>::w(L));
      launch_slab_update<R>(ne, L.N, h->q, 1.0, Bufs<R>::w(L), t2, 1, s);
      break;
    case STMG_OP_RESTRICT:
      op.restrict_to(level, t0, t2);
      break;
    case STMG_OP_PROLONG:
      launch_fill<R>(t2, (int64_t)op.ne(level - 1) * op.W(level - 1), 0.0, s);
      op.prolong_add(level - 1, t0, t2);
      break;
    default:
      fail(STMG_EINVAL, "unknown op");
  }
}

void destroy_handle(stmg_handle *h) {
  if (!h) return;
  if (h->graph_exec || h->graph_stream) {
    (void)hipStreamSynchronize(h->stream);
    drop_graph(h);
    if (h->graph_stream) (void)hipStreamDestroy(h->graph_stream);
  }
  if (!h->prof_state.recs.empty() || !h->prof_state.pool.empty()) (void)hipStreamSynchronize(h->stream);
  for (auto &r : h->prof_state.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : h->prof_state.pool) (void)hipEventDestroy(e);
  if (h->stream_ordered) {
    for (auto &b : h->bufs) (void)hipFreeAsync(b.p, h->stream);
  } else {
    for (auto &b : h->bufs) (void)hipFree(b.p);
  }
  delete h;
}

}  // namespace

namespace stmg {

hipEvent_t ProfState::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  hip_check(hipEventCreate(&e), "hipEventCreate");
  return e;
}

void Profiler::begin(hipStream_t s) {
  auto *st = static_cast<ProfState *>(impl);
  st->pending = st->get();
  hip_check(hipEventRecord(st->pending, s), "hipEventRecord");
}

void Profiler::end(hipStream_t s, const char *kernel, double flops, double bytes) {
  auto *st = static_cast<ProfState *>(impl);
  hipEvent_t b = st->get();
  hip_check(hipEventRecord(b, s), "hipEventRecord");
  st->recs.push_back({st->pending, b, kernel, flops, bytes});
  st->pending = nullptr;
}

}  // namespace stmg

namespace {
// Resolve recorded events into per-kernel sums (synchronises).
void prof_collect(stmg_handle *h) {
  ProfState &st = h->prof_state;
  if (st.recs.empty()) return;
  hip_check(hipStreamSynchronize(h->stream), "sync");
  for (auto &r : st.recs) {
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
    ProfState::Agg *g = nullptr;
    for (auto &x : st.agg)
      if (x.kernel == r.kernel) g = &x;
    if (!g) {
      st.agg.push_back({r.kernel});
      g = &st.agg.back();
    }
    g->launches++;
    g->ms += ms;
    g->flops += r.flops;
    g->bytes += r.bytes;
    st.pool.push_back(r.a);
    st.pool.push_back(r.b);
  }
  st.recs.clear();
}
}  // namespace

namespace stmg {
void alloc_point(const char *what) {
  const int64_t k = ++g_alloc_count;
  const int64_t at = g_alloc_fail_at.load();
  if (at > 0 && k == at) {
    char msg[128];
    snprintf(msg, sizeof msg, "injected allocation failure at allocation %lld (%s)", (long long)k, what);
    fail(STMG_ENOMEM, msg);
  }
}
}  // namespace stmg

// ------------------------------------------------- no-allocation scratch
// Device scratch of stmg_residual_noalloc: the internal-layout copies of x
// and b and the residual, three vectors of n_e N q doubles each. One copy
// of the array exists on every GPU the library runs on, for the life of the
// process. Host code never uses the array's name as an address: each
// device's address comes from hipGetSymbolAddress, taken once per device
// at the first setup on it.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = (size_t)8 << 20;  // 64 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// Address of `scratch` on the current device (looked up once per device).
double *scratch_address(int dev) {
  STMG_REQUIRE(dev >= 0 && dev < MAX_DEVICES, STMG_EHIP, "device id out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    STMG_REQUIRE(ptr != nullptr, STMG_EHIP, "no device address for the scratch array");
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

// ============================================================ setup phases
// Host phase: validation, topology, FP64 assembly, hierarchy (eq. (3)),
// orderings, symbolic and numeric factorisations. No HIP calls; safe to run
// on worker threads.
stmg_handle *setup_host_phase(const stmg_problem *prob, const stmg_options *opt) {
  STMG_REQUIRE(prob, STMG_EINVAL, "null argument");
  STMG_REQUIRE(prob->Nt >= 1 && (prob->Nt & (prob->Nt - 1)) == 0, STMG_EINVAL, "Nt must be a power of two");
  STMG_REQUIRE(prob->pt == 0 || prob->pt == 1, STMG_EINVAL, "pt must be 0 or 1");
  STMG_REQUIRE(prob->T > 0 && std::isfinite(prob->T), STMG_EINVAL, "T must be > 0");
  STMG_REQUIRE(prob->bc == STMG_BC_DIRICHLET || prob->bc == STMG_BC_NEUMANN, STMG_EINVAL,
               "bc must be STMG_BC_DIRICHLET or STMG_BC_NEUMANN");
  const double t0 = wall_time();
  std::unique_ptr<stmg_handle> h(new stmg_handle());
  if (opt)
    h->opt = *opt;
  else
    stmg_default_options(&h->opt);
  STMG_REQUIRE(h->opt.omega > 0 && h->opt.omega <= 1.0, STMG_EINVAL, "omega must be in (0, 1]");
  STMG_REQUIRE(smoother_sequence(h->opt.smoother) != nullptr, STMG_EINVAL, "unknown smoother sequence");
  STMG_REQUIRE(h->opt.precision == STMG_FP64 || h->opt.precision == STMG_FP32_REFINED, STMG_EINVAL,
               "unknown precision form");
  STMG_REQUIRE(h->opt.nodal >= 0 && h->opt.nodal <= STMG_NODAL_CHEBYSHEV_MAX, STMG_EINVAL,
               "nodal must be STMG_NODAL_EXACT (0) or a number of Chebyshev steps 1..16");
  STMG_REQUIRE(h->opt.slab >= 0 && h->opt.slab <= STMG_SLAB_TWOGRID_MAX, STMG_EINVAL,
               "slab must be STMG_SLAB_EXACT (0) or a number of two-grid Richardson steps 1..16");
  if (h->opt.leaf_size <= 0) h->opt.leaf_size = 8;
  STMG_REQUIRE(h->opt.gemm_rows == 0 || h->opt.gemm_rows == 32 || h->opt.gemm_rows == 64, STMG_EINVAL,
               "gemm_rows must be 0, 32 or 64");
  {
    const int c = h->opt.stream_chunk;
    STMG_REQUIRE(c == 0 || c == 1 || c == 2 || c == 4 || c == 8 || c == 16 || c == RES_CHUNK_TILES, STMG_EINVAL,
                 "stream_chunk must be 0, 1, 2, 4, 8, 16 or 32");
    STMG_REQUIRE(h->opt.row_schedule >= 0 && h->opt.row_schedule <= 3, STMG_EINVAL,
                 "row_schedule must be 0, 1, 2 or 3");
  }
  if (h->opt.max_cycles <= 0) h->opt.max_cycles = 100;
  h->pt = prob->pt;
  h->q = prob->pt + 1;
  h->Nt = prob->Nt;
  h->T = prob->T;
  h->space = build_space_levels(*prob);
  // space-time levels: halve N; coarsen space where eq. (3) holds
  LevelData L0;
  L0.mesh = 0;
  L0.N = prob->Nt;
  L0.tau = prob->T / prob->Nt;
  h->levels.push_back(std::move(L0));
  while (h->levels.back().N > 1) {
    LevelData &c = h->levels.back();
    c.lambda = h->space[c.mesh].anisotropy(c.tau);
    const bool sp = h->opt.allow_space_coarsening && c.mesh + 1 < (int32_t)h->space.size() &&
                    c.lambda >= h->opt.lambda_crit;
    LevelData n;
    n.mesh = sp ? c.mesh + 1 : c.mesh;
    n.N = c.N / 2;
    n.tau = 2.0 * c.tau;
    h->levels.push_back(std::move(n));
  }
  h->levels.back().lambda = h->space[h->levels.back().mesh].anisotropy(h->levels.back().tau);
  // meshes 0..used-1 are set up: every level's mesh, and the coarser mesh of
  // the levels with inexact slab solves
  int32_t used = h->levels.back().mesh + 1;
  for (auto &L : h->levels) {
    L.twogrid = h->opt.slab > 0 && L.N > 1 && L.mesh + 1 < (int32_t)h->space.size();
    L.fmesh = L.twogrid ? L.mesh + 1 : L.mesh;
    used = std::max(used, L.fmesh + 1);
  }
  h->mesh_slot.assign(h->space.size(), -1);
  h->meshes.resize(used);
  if (verbose()) fprintf(stderr, "[stmg] assembly and hierarchy %.2fs\n", wall_time() - t0);
  for (int32_t j = 0; j < used; ++j) {
    h->mesh_slot[j] = j;
    h->meshes[j].index = j;
    h->meshes[j].S = &h->space[j];
    setup_mesh_host(h.get(), h->meshes[j]);
    if (verbose())
      fprintf(stderr, "[stmg] mesh %d: %d edges, slab nnz(L) %.3e, %d supernodes (%.2fs)\n", j,
              h->meshes[j].S->topo.n_int_edges(), (double)h->meshes[j].sym_e.nnz_L, h->meshes[j].sym_e.ns,
              wall_time() - t0);
  }
  for (size_t l = 0; l < h->levels.size() && !dev_factor(h.get()); ++l) {
    LevelData &L = h->levels[l];
    setup_level_factor_host(h.get(), L);
    if (verbose())
      fprintf(stderr, "[stmg] level %zu (mesh %d, N %d, tau %.4g, lambda %.3g) factored (%.2fs)\n", l, L.mesh, L.N,
              L.tau, L.lambda, wall_time() - t0);
  }
  h->setup_s = wall_time() - t0;
  return h.release();
}

// Order of the slab factorisations of the device phase: largest factor
// first (ties in level order).
std::vector<size_t> factor_order(const stmg_handle *h) {
  std::vector<size_t> order(h->levels.size());
  std::iota(order.begin(), order.end(), size_t(0));
  auto entries = [&](size_t l) { return h->meshes[h->mesh_slot[h->levels[l].fmesh]].sym_e.panel_entries; };
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return entries(a) > entries(b); });
  return order;
}

// Peak device bytes of the device phase (vectors, factors, patterns, and the
// factorisation temporaries alive while the slab factors are computed, in
// factor_order before any level vector), from host data; used by the setup's
// refusal and the server's admission control. Plans and small index arrays
// are covered by a 5% margin.
int64_t estimate_device_bytes(const stmg_handle *h) {
  const bool prec = h->opt.precision == STMG_FP32_REFINED;
  int64_t bytes = 0;
  for (const auto &md : h->meshes) {
    const int64_t nnz = md.Mp.nnz(), ne = md.S->topo.n_int_edges(), nv = md.S->topo.n_int_verts();
    bytes += nnz * (4 + 8 + 8 + (prec ? 8 : 0)) + 8 * (ne + 1) + 24 * ne + 40 * nv;
    // residual row groups and LDS tiles
    const int64_t nent = (int64_t)md.gent.size() / 2;
    bytes += nent * (8 + RES_GROUP * 2 * (8 + (prec ? 4 : 0))) + 4 * (int64_t)md.gptr.size();
    bytes += 4 * (int64_t)(md.tile_ptr.size() + md.tile_cols.size()) + 2 * (int64_t)md.lcol.size();
    if (h->opt.nodal > 0) {
      bytes += md.Knp.nnz() * (4 + 8 + (prec ? 4 : 0)) + (8 + 8 + (prec ? 4 : 0)) * (nv + 1);
    } else {
      const int64_t pn = md.sym_v.panel_entries;
      bytes += pn * 8 * 2 + (prec ? pn * 4 * 2 : 0);
    }
  }
  const int64_t mesh_bytes = bytes;
  std::vector<int64_t> level_factor(h->levels.size(), 0);
  for (size_t l = 0; l < h->levels.size(); ++l) {
    const LevelData &L = h->levels[l];
    const MeshData &md = h->meshes[h->mesh_slot[L.mesh]];
    const MeshData &mf = h->meshes[h->mesh_slot[L.fmesh]];
    const int64_t W = (int64_t)L.N * h->q, ne = md.S->topo.n_int_edges(), nv = md.S->topo.n_int_verts();
    const int64_t scal = h->pt == 1 ? 16 : 8;
    const int64_t pe = mf.sym_e.panel_entries * (slab_transpose(h, L) ? 2 : 1);
    if (need64(h, L)) level_factor[l] += pe * scal;
    if (need32(h, L)) level_factor[l] += pe * scal / 2;
    bytes += level_factor[l];
    const int64_t urow = mf.sym_e.rptr[mf.sym_e.ns];
    if (L.twogrid)  // Richardson residual, smoother iterates, temporary, coarse vector, diagonals
      bytes += (prec ? 4 : 8) * W * (4 * ne + mf.S->topo.n_int_edges()) + 16 * (ne + nv);
    const bool last = l + 1 == h->levels.size();
    const int64_t nodal_extra = nv == 0 ? 0 : (h->opt.nodal > 0 ? 2 * nv : md.sym_v.rptr[md.sym_v.ns]);
    if (!prec) bytes += 8 * W * (4 * ne + urow + 2 * nv + nodal_extra);
    if (prec) {
      bytes += 4 * W * (4 * ne + urow + 2 * nv + nodal_extra);
      if (l == 0 || last) bytes += 8 * W * 3 * ne;
      if (last) bytes += 8 * W * (ne + urow);
      if (l == 0 && last) bytes += 8 * W * 2 * ne;
    }
  }
  const LevelData &L0 = h->levels[0];
  const int64_t v0 = (int64_t)h->meshes[0].S->topo.n_int_edges() * L0.N * h->q * 8;
  bytes += std::min<int64_t>((int64_t)256 << 20, 4 * v0);  // split-K workspace
  if (dev_factor(h)) {
    // factorisation temporaries (one factor at a time): front, update
    // stack, plan arrays, values and the FP64 panels of a level that keeps
    // only FP32 ones; plus rocBLAS's own workspace. The nodal factors are
    // computed with the mesh data, the slab factors after it in factor_order
    // before any level vector.
    auto factor_temp = [&](const FrontPlan &fp, const Symbolic &S, int64_t nnz, int64_t scal, bool fp64_temp) {
      return (fp.max_m2 + fp.uoff[S.ns]) * scal + 16 * (int64_t)fp.a_pos.size() + 4 * (int64_t)fp.relpos.size() +
             nnz * scal + (fp64_temp ? S.panel_entries * scal : 0) + ((int64_t)128 << 20);
    };
    int64_t peak = 0;
    for (const auto &md : h->meshes)
      if (md.S->topo.n_int_verts() > 0 && h->opt.nodal <= 0)
        peak = std::max(peak, mesh_bytes + factor_temp(md.fp_v, md.sym_v, md.S->Kn.nnz(), 8, false));
    int64_t done = mesh_bytes;
    std::vector<int64_t> temps;
    for (size_t l : factor_order(h)) {
      const LevelData &L = h->levels[l];
      const MeshData &md = h->meshes[h->mesh_slot[L.fmesh]];
      temps.push_back(factor_temp(md.fp_e, md.sym_e, md.S->M.nnz(), h->pt == 1 ? 16 : 8, !need64(h, L)));
      peak = std::max(peak, done + temps.back());
      done += level_factor[l];
    }
    if (h->factor_workers > 1) {
      // parallel factorisations: at worst every factor and the temporaries
      // of the largest factorisations, one per worker, at once
      std::sort(temps.begin(), temps.end(), std::greater<int64_t>());
      int64_t t_sum = 0;
      for (size_t i = 0; i < temps.size() && i < (size_t)h->factor_workers; ++i) t_sum += temps[i];
      peak = std::max(peak, done + t_sum);
    }
    bytes = std::max(bytes, peak);
  }
  return bytes + bytes / 20 + (1 << 20);
}

// Device phase: uploads, plans and workspaces on `stream` (no device-wide
// synchronisation, so other handles' work keeps running).
void setup_device_phase(stmg_handle *h, hipStream_t stream) {
  const double t0 = wall_time();
  h->stream = stream;
  hip_check(hipGetDevice(&h->device), "hipGetDevice");
  h->noalloc_scratch = scratch_address(h->device);
  struct RbGuard {
    stmg_handle *h;
    ~RbGuard() {
      if (h->rb) (void)rocblas_destroy_handle(h->rb);
      h->rb = nullptr;
    }
  } rb_guard{h};
  if (dev_factor(h)) {
    STMG_REQUIRE(rocblas_create_handle(&h->rb) == rocblas_status_success, STMG_EHIP, "rocblas_create_handle failed");
    STMG_REQUIRE(rocblas_set_stream(h->rb, stream) == rocblas_status_success, STMG_EHIP, "rocblas_set_stream failed");
  }
  const int32_t used = (int32_t)h->meshes.size();
  for (int32_t j = 0; j < used; ++j) {
    setup_mesh_device(h, h->meshes[j]);
    if (j > 0) setup_transfer(h, h->meshes[j - 1], h->meshes[j]);
  }
  if (verbose()) fprintf(stderr, "[stmg] mesh data and nodal factors %.2fs\n", wall_time() - t0);
  // every slab factor first, the largest first (its factorisation
  // temporaries then share the device with the mesh data and the other
  // workers' temporaries only), then the level vectors
  const std::vector<size_t> order = factor_order(h);
  const int workers = std::min<int>(h->factor_workers, (int)order.size() - 1);
  // the first (largest) factor on this thread: every kernel and library
  // routine the workers use is then loaded and initialised before they start
  for (size_t i = 0; i < order.size() && (i == 0 || workers <= 1); ++i) {
    setup_level_factor_device(h, h->levels[order[i]]);
    if (verbose())
      fprintf(stderr, "[stmg] level %zu slab factor (%s factorisation) %.2fs\n", order[i],
              dev_factor(h) ? "GPU" : "host", wall_time() - t0);
  }
  if (workers > 1) {
    // the factorisations are sequences of small dependent launches whose
    // issue dominates their time: workers with a stream and a rocBLAS handle
    // each take the next level in `order` until none is left
    std::atomic<size_t> next{1};
    std::vector<std::exception_ptr> errs(workers);
    std::vector<std::thread> pool;
    auto work = [&](int t) {
      hipStream_t st = nullptr;
      rocblas_handle rb = nullptr;
      try {
        hip_check(hipSetDevice(h->device), "hipSetDevice");
        hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
        STMG_REQUIRE(rocblas_create_handle(&rb) == rocblas_status_success, STMG_EHIP, "rocblas_create_handle failed");
        STMG_REQUIRE(rocblas_set_stream(rb, st) == rocblas_status_success, STMG_EHIP, "rocblas_set_stream failed");
        tl_setup_stream = st;
        tl_setup_rb = rb;
        for (size_t i; (i = next.fetch_add(1)) < order.size();) {
          setup_level_factor_device(h, h->levels[order[i]]);
          if (verbose())
            fprintf(stderr, "[stmg] level %zu slab factor (GPU factorisation, worker %d) %.2fs\n", order[i], t,
                    wall_time() - t0);
        }
      } catch (...) {
        errs[t] = std::current_exception();
        next.store(order.size());
      }
      tl_setup_stream = nullptr;
      tl_setup_rb = nullptr;
      if (rb) (void)rocblas_destroy_handle(rb);
      if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
      }
    };
    try {
      for (int t = 0; t < workers; ++t) pool.emplace_back(work, t);
    } catch (const std::system_error &) {
      // a thread that cannot start: the started ones (or this thread) take the rest
    }
    if (pool.empty())
      for (size_t i; (i = next.fetch_add(1)) < order.size();) setup_level_factor_device(h, h->levels[order[i]]);
    for (auto &th : pool) th.join();
    for (auto &e : errs)
      if (e) std::rethrow_exception(e);
  }
  for (size_t l = 0; l < h->levels.size(); ++l) alloc_level_vectors(h, h->levels[l], l == 0);
  // split-K partial sums of the backward solves, shared by all factors
  const LevelData &L0 = h->levels[0];
  const int64_t v0 = (int64_t)h->space[0].topo.n_int_edges() * L0.N * h->q * 8;
  const int64_t ws_bytes = std::min<int64_t>((int64_t)256 << 20, 4 * v0);
  void *ws = dev_alloc<char>(h, (size_t)ws_bytes);
  for (auto &L : h->levels) {
    L.slab.plan.splitk_ws = ws;
    L.slab.plan.splitk_bytes = ws_bytes;
  }
  for (auto &m : h->meshes) {
    m.nodal.plan.splitk_ws = ws;
    m.nodal.plan.splitk_bytes = ws_bytes;
  }
  h->n_partial = residual_blocks(h->space[0].topo.n_int_edges(), L0.N * h->q, h->q, 1) + 4096;  // any chunk
  h->d_partial = dev_alloc<double>(h, h->n_partial);
  h->d_halo = dev_alloc<double>(h, 2 * (size_t)h->space[0].topo.n_int_edges() + 64);
  h->d_scalar = dev_alloc<double>(h, GRAPH_NORM_SLOT + 1);
  hip_check(hipStreamSynchronize(stream), "setup");
  h->setup_s += wall_time() - t0;
}

namespace stmg {
namespace internal {
stmg_handle *setup_host(const stmg_problem *prob, const stmg_options *opt) { return setup_host_phase(prob, opt); }
int64_t estimate_bytes(const stmg_handle *h) { return estimate_device_bytes(h); }
void setup_device(stmg_handle *h, hipStream_t stream) { setup_device_phase(h, stream); }
void iteration(stmg_handle *h, double *dst_norm2) {
  solver_iteration(h, dst_norm2);
  check_launch();
}
// The server batches only requests of similar work per iteration (finest
// interior edge counts within a factor of 2): a batch ends when its largest
// member does, so a small request batched with a much larger one would wait
// for it every iteration.
bool batchable(const stmg_handle *a, const stmg_handle *b) {
  if (!same_cycle_shape(a, b)) return false;
  const int64_t ea = a->space[0].topo.n_int_edges(), eb = b->space[0].topo.n_int_edges();
  return ea <= 2 * eb && eb <= 2 * ea;
}
void batched_iteration(const std::vector<stmg_handle *> &hs, hipStream_t s) {
  group_iteration(hs, s, 0);
  check_launch();
}
void destroy(stmg_handle *h) { destroy_handle(h); }
const char *last_error() { return g_err.c_str(); }
}  // namespace internal
}  // namespace stmg

// =================================================================== ABI
extern "C" {

const char *stmg_strerror(int code) {
  switch (code) {
    case STMG_OK: return "ok";
    case STMG_EINVAL: return "invalid argument";
    case STMG_ENOMEM: return "out of memory";
    case STMG_ENOTCONV: return "not converged";
    case STMG_ENUMERIC: return "numerical breakdown";
    case STMG_EHIP: return "HIP runtime error";
    case STMG_EAGAIN: return "not ready";
    case STMG_ENOSYS: return "not available";
    default: return "unknown error";
  }
}

const char *stmg_last_error_message(void) { return g_err.c_str(); }

void stmg_default_options(stmg_options *o) {
  if (!o) return;
  o->omega = 0.5;
  o->lambda_crit = 0.1;
  o->allow_space_coarsening = 1;
  o->smoother = STMG_SMOOTH_SAS;
  o->precision = STMG_FP64;
  o->rtol = 1e-8;
  o->max_cycles = 100;
  o->host_only = 0;
  o->stream_chunk = 0;
  o->row_schedule = 0;
  o->leaf_size = 8;
  o->gemm_rows = 0;
  o->factor_transpose = -1;
  o->gemm_splitk = 0;
  o->device_factor = -1;
  o->nodal = STMG_NODAL_EXACT;
  o->graph = 1;
  o->slab = STMG_SLAB_EXACT;
}

int stmg_setup(const stmg_problem *prob, const stmg_options *opt, void *stream, stmg_handle **out) {
  if (out) *out = nullptr;
  stmg_handle *h = nullptr;
  int rc = guard([&] {
    STMG_REQUIRE(out, STMG_EINVAL, "null argument");
    h = setup_host_phase(prob, opt);
    if (!h->opt.host_only) {
      int ndev = 0;
      hip_check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
      STMG_REQUIRE(ndev > 0, STMG_EHIP, "no HIP device");
      // refuse before allocating when the device cannot hold the handle
      size_t free_b = 0, total_b = 0;
      hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
      // parallel GPU factorisations, as many as their temporaries fit (at
      // most STMG_SETUP_THREADS from the environment; 1 = one stream)
      if (dev_factor(h) && !h->stream_ordered)
        for (h->factor_workers = setup_threads_limit();
             h->factor_workers > 1 && estimate_device_bytes(h) > (int64_t)free_b; h->factor_workers /= 2) {
        }
      const int64_t need = estimate_device_bytes(h);
      if (need > (int64_t)free_b) {
        char msg[160];
        snprintf(msg, sizeof msg, "the handle needs about %.1f GB of device memory, %.1f GB are free",
                 need / 1e9, free_b / 1e9);
        fail(STMG_ENOMEM, msg);
      }
      if (verbose()) fprintf(stderr, "[stmg] estimated device bytes %.2f GB (free %.2f GB)\n", need / 1e9, free_b / 1e9);
      setup_device_phase(h, static_cast<hipStream_t>(stream));
    }
  });
  if (rc != STMG_OK) {
    destroy_handle(h);
    return rc;
  }
  *out = h;
  return STMG_OK;
}

void stmg_destroy(stmg_handle *h) { destroy_handle(h); }

int stmg_info(const stmg_handle *h, stmg_info_t *info) {
  return guard([&] {
    STMG_REQUIRE(h && info, STMG_EINVAL, "null argument");
    info->n_edges = h->space[0].topo.ne;
    info->n_levels = (int32_t)h->levels.size();
    info->pt = h->pt;
    info->device_bytes = h->device_bytes;
    info->factor_bytes = h->factor_bytes;
  });
}

int stmg_level_info(const stmg_handle *h, int32_t level, stmg_level_info_t *info) {
  return guard([&] {
    STMG_REQUIRE(h && info, STMG_EINVAL, "null argument");
    STMG_REQUIRE(level >= 0 && level < (int32_t)h->levels.size(), STMG_EINVAL, "level out of range");
    const LevelData &L = h->levels[level];
    const MeshData &md = h->meshes[h->mesh_slot[L.mesh]];
    const MeshData &mf = h->meshes[h->mesh_slot[L.fmesh]];
    info->mesh = L.mesh;
    info->N = L.N;
    info->tau = L.tau;
    info->n_e = md.S->topo.n_int_edges();
    info->n_v = md.S->topo.n_int_verts();
    info->nnz_pattern = md.S->M.nnz();
    info->factor_nnz_slab = mf.sym_e.nnz_L;
    info->factor_nnz_nodal = md.sym_v.nnz_L;
    info->n_supernodes_slab = mf.sym_e.ns;
    info->lambda = L.lambda;
    info->factor_nnz_slab_struct = mf.sym_e.nnz_L_struct;
    info->factor_nnz_nodal_struct = md.sym_v.nnz_L_struct;
    info->slab_factor_mesh = L.fmesh;
    info->slab_steps = L.twogrid ? h->opt.slab : 0;
  });
}

int stmg_edges(const stmg_handle *h, int32_t *n_edges, const int32_t **edge_vertices) {
  return guard([&] {
    STMG_REQUIRE(h && n_edges && edge_vertices, STMG_EINVAL, "null argument");
    *n_edges = h->space[0].topo.ne;
    *edge_vertices = h->space[0].topo.edges.data();
  });
}

int stmg_load(stmg_handle *h, const double *rhs_dev, const double *u0_dev, const double *x0_dev,
              double *bnorm) {
  return guard([&] {
    require_device(h);
    STMG_REQUIRE(rhs_dev, STMG_EINVAL, "rhs is null");
    Ops op{h, h->stream};
    LevelData &L = h->levels[0];
    MeshData &md = op.mesh(0);
    const int32_t ne = op.ne(0), E = md.S->topo.ne;
    launch_abi_to_internal(ne, L.N, h->q, E, md.d_map_abi, rhs_dev, L.b, h->stream);
    if (u0_dev)
      launch_fold_initial(ne, L.N, h->q, md.d_ptr, md.d_col, md.d_mval, md.d_map_abi, u0_dev, L.b, h->stream);
    if (x0_dev)
      launch_abi_to_internal(ne, L.N, h->q, E, md.d_map_abi, x0_dev, L.x, h->stream);
    else
      launch_fill(L.x, (int64_t)ne * op.W(0), 0.0, h->stream);
    const int nb = launch_sumsq(L.b, (int64_t)ne * op.W(0), h->d_partial, h->stream);
    launch_sum(h->d_partial, nb, h->d_scalar, h->stream);
    // the precision form refines from the FP64 residual of the current iterate
    if (h->opt.precision == STMG_FP32_REFINED) op.residual(0, L.x, L.b, L.w, RES_OUT_R, nullptr);
    check_launch();
    double b2 = 0.0;
    hip_check(hipMemcpyAsync(&b2, h->d_scalar, sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy");
    hip_check(hipStreamSynchronize(h->stream), "sync");
    STMG_REQUIRE(std::isfinite(b2), STMG_ENUMERIC, "non-finite right-hand side");
    h->bnorm = std::sqrt(b2);
    h->history.clear();
    h->cycles = 0;
    if (bnorm) *bnorm = h->bnorm;
  });
}

int stmg_cycles(stmg_handle *h, int32_t n_cycles, double *res_host) {
  return guard([&] {
    require_device(h);
    STMG_REQUIRE(n_cycles >= 0 && n_cycles <= 8192, STMG_EINVAL, "n_cycles out of range");
    for (int32_t i = 0; i < n_cycles; ++i) run_iteration(h, h->d_scalar + i);
    check_launch();
    if (res_host && n_cycles > 0) {
      std::vector<double> r2(n_cycles);
      hip_check(hipMemcpyAsync(r2.data(), h->d_scalar, n_cycles * sizeof(double), hipMemcpyDeviceToHost,
                               h->stream),
                "copy");
      hip_check(hipStreamSynchronize(h->stream), "sync");
      for (int32_t i = 0; i < n_cycles; ++i) {
        res_host[i] = std::sqrt(r2[i]) / (h->bnorm > 0 ? h->bnorm : 1.0);
        h->history.push_back(res_host[i]);
      }
    }
    h->cycles += n_cycles;
  });
}

int stmg_cycles_batched(stmg_handle *const *hs, int32_t n, int32_t n_cycles, double *res_host) {
  return guard([&] {
    STMG_REQUIRE(hs && n >= 1 && n <= SOLVE_GROUP_MAX, STMG_EINVAL, "need 1 to 8 handles");
    STMG_REQUIRE(n_cycles >= 0 && n_cycles <= 8192, STMG_EINVAL, "n_cycles out of range");
    std::vector<stmg_handle *> v(hs, hs + n);
    for (int32_t i = 0; i < n; ++i) {
      require_device(v[i]);
      STMG_REQUIRE(same_cycle_shape(v[0], v[i]), STMG_EINVAL,
                   "batched handles need the same N_t, p_t, precision form and smoother");
      for (int32_t j = 0; j < i; ++j) STMG_REQUIRE(v[j] != v[i], STMG_EINVAL, "a handle appears twice");
    }
    // the members' own streams first finish what they hold
    for (auto *h : v) hip_check(hipStreamSynchronize(h->stream), "sync");
    hipStream_t s = v[0]->stream;
    for (int32_t c = 0; c < n_cycles; ++c) group_iteration(v, s, c);
    check_launch();
    if (n_cycles > 0) {
      std::vector<double> r2((size_t)n * n_cycles);
      for (int32_t i = 0; i < n; ++i)
        hip_check(hipMemcpyAsync(r2.data() + (size_t)i * n_cycles, v[i]->d_scalar, n_cycles * sizeof(double),
                                 hipMemcpyDeviceToHost, s),
                  "copy");
      hip_check(hipStreamSynchronize(s), "sync");
      for (int32_t i = 0; i < n; ++i)
        for (int32_t c = 0; c < n_cycles; ++c) {
          const double rel = std::sqrt(r2[(size_t)i * n_cycles + c]) / (v[i]->bnorm > 0 ? v[i]->bnorm : 1.0);
          v[i]->history.push_back(rel);
          if (res_host) res_host[(size_t)i * n_cycles + c] = rel;
        }
    }
    for (auto *h : v) h->cycles += n_cycles;
  });
}

int stmg_power_rate(stmg_handle *h, const double *x0_dev, int32_t max_cycles, double underflow, double *rate,
                    double *rates_host, int32_t *n_done) {
  return guard([&] {
    require_device(h);
    STMG_REQUIRE(x0_dev && rate, STMG_EINVAL, "x0 or rate is null");
    STMG_REQUIRE(max_cycles >= 1 && max_cycles <= 8192, STMG_EINVAL, "max_cycles out of range");
    STMG_REQUIRE(std::isfinite(underflow) && underflow >= 0.0 && underflow < 1.0, STMG_EINVAL,
                 "underflow must be in [0, 1)");
    STMG_REQUIRE(h->opt.precision == STMG_FP64, STMG_EINVAL, "the power iteration runs in the FP64 form");
    Ops op{h, h->stream};
    LevelData &L = h->levels[0];
    MeshData &md = op.mesh(0);
    const int32_t ne = op.ne(0), E = md.S->topo.ne;
    const int64_t n = (int64_t)ne * op.W(0);
    launch_fill(L.b, n, 0.0, h->stream);
    launch_abi_to_internal(ne, L.N, h->q, E, md.d_map_abi, x0_dev, L.x, h->stream);
    h->bnorm = 0.0;
    h->history.clear();
    h->cycles = 0;
    auto norm2 = [&](double *dst) {
      const int nb = launch_sumsq(L.x, n, h->d_partial, h->stream);
      launch_sum(h->d_partial, nb, dst, h->stream);
    };
    // cycles run in batches between host reads of their norms
    constexpr int32_t BATCH = 64;
    std::vector<double> n2(BATCH);
    norm2(h->d_scalar);
    check_launch();
    hip_check(hipMemcpyAsync(n2.data(), h->d_scalar, sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy");
    hip_check(hipStreamSynchronize(h->stream), "sync");
    const double start = std::sqrt(n2[0]);
    STMG_REQUIRE(std::isfinite(start), STMG_ENUMERIC, "non-finite x0");
    STMG_REQUIRE(start > 0.0, STMG_EINVAL, "x0 is zero on the interior edges");
    double prev = start, best = 0.0;
    int32_t done = 0;
    bool stop = false;
    while (!stop && done < max_cycles) {
      const int32_t nbat = std::min(BATCH, max_cycles - done);
      for (int32_t i = 0; i < nbat; ++i) {
        op.vcycle(0, L.x, L.b);
        norm2(h->d_scalar + i);
      }
      check_launch();
      hip_check(hipMemcpyAsync(n2.data(), h->d_scalar, nbat * sizeof(double), hipMemcpyDeviceToHost, h->stream),
                "copy");
      hip_check(hipStreamSynchronize(h->stream), "sync");
      for (int32_t i = 0; i < nbat && !stop; ++i) {
        const double nx = std::sqrt(n2[i]);
        STMG_REQUIRE(std::isfinite(nx), STMG_ENUMERIC, "non-finite iterate in the power iteration");
        const double r = nx / prev;
        if (rates_host) rates_host[done] = r;
        best = std::max(best, r);
        prev = nx;
        ++done;
        stop = nx < underflow * start;
      }
    }
    h->cycles = done;
    *rate = best;
    if (n_done) *n_done = done;
  });
}

int stmg_store(stmg_handle *h, double *x_dev) {
  return guard([&] {
    require_device(h);
    STMG_REQUIRE(x_dev, STMG_EINVAL, "x is null");
    Ops op{h, h->stream};
    MeshData &md = op.mesh(0);
    const int32_t E = md.S->topo.ne;
    launch_fill(x_dev, (int64_t)E * op.W(0), 0.0, h->stream);
    launch_internal_to_abi(op.ne(0), h->levels[0].N, h->q, E, md.d_map_abi, h->levels[0].x, x_dev, h->stream);
    check_launch();
  });
}

int stmg_vcycle(stmg_handle *h, const double *rhs_dev, double *x_dev) {
  return guard([&] {
    require_device(h);
    STMG_REQUIRE(rhs_dev && x_dev, STMG_EINVAL, "null argument");
    Ops op{h, h->stream};
    LevelData &L = h->levels[0];
    MeshData &md = op.mesh(0);
    const int32_t ne = op.ne(0), E = md.S->topo.ne;
    launch_abi_to_internal(ne, L.N, h->q, E, md.d_map_abi, rhs_dev, L.b, h->stream);
    launch_abi_to_internal(ne, L.N, h->q, E, md.d_map_abi, x_dev, L.x, h->stream);
    if (h->opt.precision == STMG_FP32_REFINED) {
      // the refinement step starts from the FP64 residual of the iterate
      op.residual(0, L.x, L.b, L.w, RES_OUT_R, nullptr);
      OpsT<float> o32{h, h->stream};
      const int64_t n = (int64_t)ne * op.W(0);
      launch_to_float(n, L.w, L.b32, h->stream);
      launch_fill<float>(L.x32, n, 0.0, h->stream);
      o32.vcycle(0, L.x32, L.b32);
      launch_add_float(n, L.x32, L.x, h->stream);
    } else {
      op.vcycle(0, L.x, L.b);
    }
    launch_fill(x_dev, (int64_t)E * op.W(0), 0.0, h->stream);
    launch_internal_to_abi(ne, L.N, h->q, E, md.d_map_abi, L.x, x_dev, h->stream);
    check_launch();
  });
}

int64_t stmg_debug_fail_alloc(int64_t k) {
  const int64_t n = g_alloc_count.exchange(0);
  g_alloc_fail_at.store(k > 0 ? k : 0);
  return n;
}

int stmg_solve(stmg_handle *h, const double *rhs_dev, const double *u0_dev, const double *x0_dev,
               double *x_dev, stmg_report *rep) {
  int status = STMG_OK;
  int rc = guard([&] {
    require_device(h);
    const double t0 = wall_time();
    double bn = 0.0;
    int e = stmg_load(h, rhs_dev, u0_dev, x0_dev, &bn);
    if (e != STMG_OK) fail(e, g_err);
    h->history.clear();
    h->rel_res = 0.0;
    h->cycles = 0;
    if (bn > 0.0) {
      status = STMG_ENOTCONV;
      for (int32_t c = 0; c < h->opt.max_cycles; ++c) {
        run_iteration(h, h->d_scalar);
        check_launch();
        double r2 = 0.0;
        hip_check(hipMemcpyAsync(&r2, h->d_scalar, sizeof(double), hipMemcpyDeviceToHost, h->stream), "copy");
        hip_check(hipStreamSynchronize(h->stream), "sync");
        ++h->cycles;
        h->rel_res = std::sqrt(r2) / bn;
        h->history.push_back(h->rel_res);
        if (!std::isfinite(h->rel_res)) {
          status = STMG_ENUMERIC;
          break;
        }
        if (h->rel_res <= h->opt.rtol) {
          status = STMG_OK;
          break;
        }
      }
    }
    e = stmg_store(h, x_dev);
    if (e != STMG_OK) fail(e, g_err);
    hip_check(hipStreamSynchronize(h->stream), "sync");
    h->solve_s = wall_time() - t0;
    if (rep) {
      rep->cycles = h->cycles;
      rep->rel_res = h->rel_res;
      rep->setup_s = h->setup_s;
      rep->solve_s = h->solve_s;
      rep->res_history = h->history.data();
    }
  });
  if (rc != STMG_OK) return rc;
  if (status == STMG_ENOTCONV) g_err = "max_cycles reached before rtol";
  if (status == STMG_ENUMERIC) g_err = "non-finite residual";
  return status;
}

int stmg_residual(stmg_handle *h, const double *x_dev, const double *rhs_dev, const double *u0_dev,
                  double *r_dev) {
  return guard([&] {
    require_device(h);
    STMG_REQUIRE(x_dev && rhs_dev && r_dev, STMG_EINVAL, "null argument");
    Ops op{h, h->stream};
    LevelData &L = h->levels[0];
    MeshData &md = op.mesh(0);
    const int32_t ne = op.ne(0), E = md.S->topo.ne;
    double *tb = tmp_buf(h, 0), *tx = tmp_buf(h, 1), *tr = tmp_buf(h, 2);
    launch_abi_to_internal(ne, L.N, h->q, E, md.d_map_abi, rhs_dev, tb, h->stream);
    if (u0_dev)
      launch_fold_initial(ne, L.N, h->q, md.d_ptr, md.d_col, md.d_mval, md.d_map_abi, u0_dev, tb, h->stream);
    launch_abi_to_internal(ne, L.N, h->q, E, md.d_map_abi, x_dev, tx, h->stream);
    op.residual(0, tx, tb, tr, RES_OUT_R, nullptr);
    launch_fill(r_dev, (int64_t)E * op.W(0), 0.0, h->stream);
    launch_internal_to_abi(ne, L.N, h->q, E, md.d_map_abi, tr, r_dev, h->stream);
    check_launch();
    hip_check(hipStreamSynchronize(h->stream), "sync");
  });
}

int stmg_residual_noalloc(stmg_handle *h, const double *x_dev, const double *rhs_dev, const double *u0_dev,
                          double *r_dev) {
  return guard([&] {
    require_device(h);
    STMG_REQUIRE(x_dev && rhs_dev && r_dev, STMG_EINVAL, "null argument");
    STMG_REQUIRE(h->noalloc_scratch, STMG_EHIP, "no scratch address for the handle's device");
    int cur = -1;
    hip_check(hipGetDevice(&cur), "hipGetDevice");
    STMG_REQUIRE(cur == h->device, STMG_EINVAL, "the handle's device is not the current device");
    Ops op{h, h->stream};
    LevelData &L = h->levels[0];
    MeshData &md = op.mesh(0);
    const int32_t ne = op.ne(0), E = md.S->topo.ne;
    const size_t n = (size_t)ne * op.W(0);
    if (3 * n > NOALLOC_SCRATCH_DOUBLES) {
      char msg[160];
      snprintf(msg, sizeof msg, "problem too large for the no-allocation residual: 3 x %zu values, limit %zu",
               n, NOALLOC_SCRATCH_DOUBLES);
      fail(STMG_EINVAL, msg);
    }
    double *tb = h->noalloc_scratch, *tx = tb + n, *tr = tx + n;
    launch_abi_to_internal(ne, L.N, h->q, E, md.d_map_abi, rhs_dev, tb, h->stream);
    if (u0_dev)
      launch_fold_initial(ne, L.N, h->q, md.d_ptr, md.d_col, md.d_mval, md.d_map_abi, u0_dev, tb, h->stream);
    launch_abi_to_internal(ne, L.N, h->q, E, md.d_map_abi, x_dev, tx, h->stream);
    op.residual(0, tx, tb, tr, RES_OUT_R, nullptr);
    launch_fill(r_dev, (int64_t)E * op.W(0), 0.0, h->stream);
    launch_internal_to_abi(ne, L.N, h->q, E, md.d_map_abi, tr, r_dev, h->stream);
    check_launch();
  });
}

int stmg_level_apply(stmg_handle *h, int32_t level, int32_t op_code, const double *in_dev,
                     const double *in2_dev, double *out_dev) {
  return guard([&] {
    require_device(h);
    const int32_t nl = (int32_t)h->levels.size();
    STMG_REQUIRE(level >= 0 && level < nl, STMG_EINVAL, "level out of range");
    STMG_REQUIRE(in_dev && out_dev, STMG_EINVAL, "null argument");
    STMG_REQUIRE(op_code >= STMG_OP_RESIDUAL && op_code <= STMG_OP_VCYCLE, STMG_EINVAL, "unknown op");
    const bool needs_in2 = op_code == STMG_OP_RESIDUAL || op_code == STMG_OP_SMOOTH_S ||
                           op_code == STMG_OP_NODAL_A || op_code == STMG_OP_SAS || op_code == STMG_OP_VCYCLE;
    STMG_REQUIRE(!needs_in2 || in2_dev, STMG_EINVAL, "in2 is null");
    STMG_REQUIRE(op_code != STMG_OP_RESTRICT || level + 1 < nl, STMG_EINVAL, "no coarser level");
    STMG_REQUIRE(op_code != STMG_OP_PROLONG || level >= 1, STMG_EINVAL, "no finer level");
    const bool prec = h->opt.precision == STMG_FP32_REFINED;
    const bool last = level + 1 == nl;
    STMG_REQUIRE(!(prec && last && (op_code == STMG_OP_SMOOTH_S || op_code == STMG_OP_NODAL_A || op_code == STMG_OP_SAS)),
                 STMG_ENOSYS, "the precision form only solves exactly on the coarsest level");
    Ops op{h, h->stream};
    hipStream_t s = h->stream;
    MeshData &md = op.mesh(level);
    const int32_t n = op.ne(level);
    const int out_level = op_code == STMG_OP_RESTRICT ? level + 1 : (op_code == STMG_OP_PROLONG ? level - 1 : level);
    const int64_t n_in = (int64_t)n * op.W(level), n_out = (int64_t)op.ne(out_level) * op.W(out_level);
    double *t0 = tmp_buf(h, 0), *t1 = tmp_buf(h, 1), *t2 = tmp_buf(h, 2);
    launch_abi_to_internal(n, h->levels[level].N, h->q, n, md.d_map_level, in_dev, t0, s);
    if (needs_in2) launch_abi_to_internal(n, h->levels[level].N, h->q, n, md.d_map_level, in2_dev, t1, s);
    // the slab solve of the precision form's coarsest level is its FP64 solve
    if (!prec || (last && op_code == STMG_OP_SLAB_SOLVE)) {
      apply_op<double>(h, level, op_code, t0, t1, t2);
    } else {
      float *f0 = tmp_buf32(h, 0), *f1 = tmp_buf32(h, 1), *f2 = tmp_buf32(h, 2);
      launch_to_float(n_in, t0, f0, s);
      if (needs_in2) launch_to_float(n_in, t1, f1, s);
      apply_op<float>(h, level, op_code, f0, f1, f2);
      launch_to_double(n_out, f2, t2, s);
    }
    MeshData &mo = op.mesh(out_level);
    const int32_t no = op.ne(out_level);
    launch_internal_to_abi(no, h->levels[out_level].N, h->q, no, mo.d_map_level, t2, out_dev, s);
    check_launch();
    hip_check(hipStreamSynchronize(s), "sync");
  });
}

int stmg_export_matrix(const stmg_handle *h, int32_t level, int32_t which, int32_t *n_rows, int32_t *n_cols,
                       int64_t *nnz, int64_t *row_ptr, int32_t *col, double *val) {
  return guard([&] {
    STMG_REQUIRE(h && n_rows && n_cols && nnz, STMG_EINVAL, "null argument");
    STMG_REQUIRE(level >= 0 && level < (int32_t)h->levels.size(), STMG_EINVAL, "level out of range");
    const SpaceLevel &S = h->space[h->levels[level].mesh];
    const Csr *A = nullptr;
    switch (which) {
      case 0: A = &S.M; break;
      case 1: A = &S.K; break;
      case 2: A = &S.G; break;
      case 3: A = &S.Kn; break;
      case 4:
        STMG_REQUIRE(h->levels[level].mesh > 0, STMG_EINVAL, "level uses the finest mesh: no P_e");
        A = &S.Pe;
        break;
      default: fail(STMG_EINVAL, "unknown matrix");
    }
    *n_rows = A->n_rows;
    *n_cols = A->n_cols;
    *nnz = A->nnz();
    if (row_ptr) std::copy(A->ptr.begin(), A->ptr.end(), row_ptr);
    if (col) std::copy(A->col.begin(), A->col.end(), col);
    if (val) std::copy(A->val.begin(), A->val.end(), val);
  });
}

int stmg_set_stream_tuning(stmg_handle *h, int32_t stream_chunk, int32_t row_schedule) {
  return guard([&] {
    STMG_REQUIRE(h, STMG_EINVAL, "null handle");
    const int c = stream_chunk;
    STMG_REQUIRE(c == 0 || c == 1 || c == 2 || c == 4 || c == 8 || c == 16 || c == RES_CHUNK_TILES, STMG_EINVAL,
                 "stream_chunk must be 0, 1, 2, 4, 8, 16 or 32");
    STMG_REQUIRE(row_schedule >= 0 && row_schedule <= 3, STMG_EINVAL, "row_schedule must be 0, 1, 2 or 3");
    STMG_REQUIRE(row_schedule == 1 || (row_schedule == 3) != h->rows_hilbert, STMG_EINVAL,
                 "row_schedule needs the space-filling curve chosen at setup");
    h->opt.stream_chunk = stream_chunk;
    h->opt.row_schedule = row_schedule;
    if (h->graph_exec) {  // the captured launches used the old shape
      hip_check(hipStreamSynchronize(h->stream), "sync");
      drop_graph(h);
    }
  });
}

int stmg_profile(stmg_handle *h, int32_t enable) {
  return guard([&] {
    require_device(h);
    prof_collect(h);
    h->prof.impl = &h->prof_state;
    h->prof_state.agg.clear();
    h->prof_state.on = enable != 0;
    set_profiler(h, h->prof_state.on);
  });
}

int stmg_profile_count(stmg_handle *h, int32_t *n_kernels) {
  return guard([&] {
    require_device(h);
    STMG_REQUIRE(n_kernels, STMG_EINVAL, "null argument");
    prof_collect(h);
    *n_kernels = (int32_t)h->prof_state.agg.size();
  });
}

int stmg_profile_get(stmg_handle *h, int32_t i, char *name, int32_t name_len, int64_t *launches,
                     double *total_ms, double *flops, double *bytes) {
  return guard([&] {
    require_device(h);
    prof_collect(h);
    STMG_REQUIRE(i >= 0 && i < (int32_t)h->prof_state.agg.size(), STMG_EINVAL, "kernel index out of range");
    const auto &g = h->prof_state.agg[i];
    if (name && name_len > 0) {
      snprintf(name, (size_t)name_len, "%s", g.kernel.c_str());
    }
    if (launches) *launches = g.launches;
    if (total_ms) *total_ms = g.ms;
    if (flops) *flops = g.flops;
    if (bytes) *bytes = g.bytes;
  });
}

int stmg_export_factor(const stmg_handle *h, int32_t level, int32_t which, int32_t *n, int32_t *ns,
                       int64_t *n_rows_total, int64_t *n_panel, int32_t *is_complex, int32_t *perm,
                       int32_t *col0, int64_t *rptr, int32_t *rows, int64_t *panel_off, double *panel) {
  return guard([&] {
    STMG_REQUIRE(h && n && ns && n_rows_total && n_panel && is_complex, STMG_EINVAL, "null argument");
    STMG_REQUIRE(level >= 0 && level < (int32_t)h->levels.size(), STMG_EINVAL, "level out of range");
    const LevelData &L = h->levels[level];
    const MeshData &md = h->meshes[h->mesh_slot[L.mesh]];
    const MeshData &mf = h->meshes[h->mesh_slot[L.fmesh]];  // of the slab factor the level keeps
    const Symbolic *S = nullptr;
    const std::vector<int64_t> *off = nullptr;
    const double *vals = nullptr;
    size_t nvals = 0;
    int cpx = 0;
    std::vector<double> copy;  // device panels copied back
    if (!h->opt.host_only) {
      STMG_REQUIRE(which == 0 || which == 1, STMG_EINVAL, "which must be 0 or 1");
      const DevFactor &D = which == 0 ? L.slab : md.nodal;
      S = which == 0 ? &mf.sym_e : &md.sym_v;
      STMG_REQUIRE(D.f.panel != nullptr && !D.h_panel_off.empty(), STMG_ENOSYS,
                   "no FP64 factor of this level on the device");
      cpx = which == 0 && D.is_complex ? 1 : 0;
      off = &D.h_panel_off;
      nvals = (size_t)D.h_panel_off[S->ns] * (cpx ? 2 : 1);
      if (panel) {
        copy.resize(nvals);
        hip_check(hipMemcpyAsync(copy.data(), D.f.panel, nvals * sizeof(double), hipMemcpyDeviceToHost,
                                 h->stream),
                  "copy");
        hip_check(hipStreamSynchronize(h->stream), "copy");
        vals = copy.data();
      }
    } else if (which == 0) {
      S = &mf.sym_e;
      if (L.slab_host_c) {
        off = &L.slab_host_c->panel_off;
        vals = reinterpret_cast<const double *>(L.slab_host_c->panel.data());
        nvals = 2 * L.slab_host_c->panel.size();
        cpx = 1;
      } else {
        STMG_REQUIRE(L.slab_host_r != nullptr, STMG_EINVAL, "no slab factor");
        off = &L.slab_host_r->panel_off;
        vals = L.slab_host_r->panel.data();
        nvals = L.slab_host_r->panel.size();
      }
    } else if (which == 1) {
      STMG_REQUIRE(md.nodal_host != nullptr, STMG_EINVAL, "no nodal factor");
      S = &md.sym_v;
      off = &md.nodal_host->panel_off;
      vals = md.nodal_host->panel.data();
      nvals = md.nodal_host->panel.size();
    } else {
      fail(STMG_EINVAL, "which must be 0 or 1");
    }
    *n = S->n;
    *ns = S->ns;
    *n_rows_total = (int64_t)S->rows.size();
    *n_panel = (int64_t)(*off)[S->ns];
    *is_complex = cpx;
    if (perm) std::copy(S->perm.begin(), S->perm.end(), perm);
    if (col0) std::copy(S->col0.begin(), S->col0.end(), col0);
    if (rptr) std::copy(S->rptr.begin(), S->rptr.end(), rptr);
    if (rows) std::copy(S->rows.begin(), S->rows.end(), rows);
    if (panel_off) std::copy(off->begin(), off->end(), panel_off);
    if (panel) std::copy(vals, vals + nvals, panel);
  });
}

}  // extern "C"
