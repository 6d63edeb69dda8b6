// Handle state of the stmg library: per-mesh and per-level host and device
// data, and the V-cycle driver.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "factor.hpp"
#include "factor_dev.hpp"
#include "kernels.hpp"
#include "ordering.hpp"
#include "space.hpp"

namespace stmg {

// Device allocation owned by a handle.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Device copy of one factor plus its solve plan.
struct DevFactor {
  bool is_complex = false;
  FactorDev f{};                 // FP64 panels (null when only FP32 is kept)
  FactorDev f32{};               // FP32 panels of the precision form (same plan)
  SolvePlan plan{};
  int64_t u_rows = 0;            // sum of r_s
  int64_t factor_bytes = 0;
  std::vector<int64_t> h_panel_off;  // panel offsets (host copy)
  // host-side plan storage (descriptors point into device arrays)
  std::vector<int64_t> h_tgt_off, h_src_off, h_xtgt_end, h_xsrc_end;
  std::vector<SolvePlan::Launch> fwd, bwd;
};

struct MeshData {
  int32_t index = 0;
  SpaceLevel *S = nullptr;
  NdTree nd;
  Symbolic sym_e, sym_v;
  FrontPlan fp_e, fp_v;          // assembly plans of the device factorisation
  Csr Mp, Kp;                    // M, K in factor (internal) numbering
  std::vector<int32_t> sched;    // residual visiting order of the internal rows
  std::vector<int32_t> tile_ptr, tile_cols;  // residual LDS tiles (see ResidualArgsT)
  std::vector<uint16_t> lcol;
  int32_t tile_union_max = 0, tile_nnz_max = 0;
  std::vector<int32_t> gptr, gent;  // residual row groups (see ResidualArgsT)
  std::vector<double> gval;
  // device
  int64_t *d_ptr = nullptr;
  int32_t *d_sched = nullptr;
  int32_t *d_tile_ptr = nullptr, *d_tile_cols = nullptr;
  uint16_t *d_lcol = nullptr;
  int32_t *d_gptr = nullptr, *d_gent = nullptr;
  double *d_gval = nullptr;
  float *d_gval32 = nullptr;
  int32_t *d_col = nullptr;
  double *d_mval = nullptr, *d_kval = nullptr;
  float *d_mval32 = nullptr, *d_kval32 = nullptr;
  int32_t *d_head = nullptr, *d_tail = nullptr;  // G: edge -> vertex (internal), -1 boundary
  int64_t *d_gt_ptr = nullptr;                   // G^T CSR over internal vertices
  int32_t *d_gt_edge = nullptr;
  int8_t *d_gt_sign = nullptr;
  int32_t *d_map_level = nullptr;  // internal edge row -> ascending interior index
  int32_t *d_map_abi = nullptr;    // internal edge row -> global edge id (mesh 0)
  // transfer from the finer mesh (index-1) to this one, internal numberings
  int64_t *d_pt_ptr = nullptr;     // P_e^T rows (this mesh's edges)
  int32_t *d_pt_col = nullptr;
  double *d_pt_val = nullptr;
  int64_t *d_p_ptr = nullptr;      // P_e rows (finer mesh's edges)
  int32_t *d_p_col = nullptr;
  double *d_p_val = nullptr;
  std::unique_ptr<HostFactor<double>> nodal_host;
  DevFactor nodal;
  // inexact nodal solves (option nodal > 0): K_n in the internal vertex
  // numbering, its inverse diagonal and the Gershgorin bound of D^{-1} K_n
  Csr Knp;
  double kn_lmax = 0.0;
  int64_t *d_kn_ptr = nullptr;
  int32_t *d_kn_col = nullptr;
  double *d_kn_val = nullptr, *d_kn_dinv = nullptr;
  float *d_kn_val32 = nullptr, *d_kn_dinv32 = nullptr;
};

struct LevelData {
  int32_t mesh = 0, N = 0;
  double tau = 0.0;
  double lambda = 0.0;
  // inexact slab solves (option slab = k > 0, levels with N > 1 whose mesh
  // has a coarser one): the slab factor below is then the one of the coarser
  // mesh fmesh = mesh + 1 with this level's tau
  bool twogrid = false;
  int32_t fmesh = 0;
  std::unique_ptr<HostFactor<double>> slab_host_r;
  std::unique_ptr<HostFactor<cplx>> slab_host_c;
  DevFactor slab;
  // device vectors (internal layout): FP64, and FP32 for the precision form
  double *x = nullptr, *b = nullptr, *w = nullptr, *z = nullptr, *u = nullptr;
  double *g = nullptr, *zn = nullptr, *un = nullptr;
  float *x32 = nullptr, *b32 = nullptr, *w32 = nullptr, *z32 = nullptr, *u32 = nullptr;
  float *g32 = nullptr, *zn32 = nullptr, *un32 = nullptr;
  double *yn = nullptr;          // second iterate buffer of the inexact nodal solve
  float *yn32 = nullptr;
  // two-grid slab solves: diag(A)^{-1} per internal edge and diag(mu K_n)^{-1}
  // per internal vertex (complex for DG degree 1), the Richardson residual,
  // two smoother iterates, a residual temporary (n_e x W values each) and the
  // coarse vector (coarse n_e x W)
  double *tg_dinv = nullptr, *tg_dn = nullptr;
  double *tg_r = nullptr, *tg_a = nullptr, *tg_b = nullptr, *tg_t = nullptr, *tg_c = nullptr;
  float *tg_dinv32 = nullptr, *tg_dn32 = nullptr;  // the precision form's (FP32 smoother)
  float *tg_r32 = nullptr, *tg_a32 = nullptr, *tg_b32 = nullptr, *tg_t32 = nullptr, *tg_c32 = nullptr;
  // precision form with one level (N_t = 1): the FP64 coarsest solve's own
  // iterate and right-hand side, apart from the outer x and b of level 0
  double *xe = nullptr, *be = nullptr;
};

// Event-pair timing of individual launches (see Profiler).
struct ProfRecord {
  hipEvent_t a, b;
  std::string kernel;
  double flops, bytes;
};
struct ProfState {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<ProfRecord> recs;
  hipEvent_t pending = nullptr;
  struct Agg {
    std::string kernel;
    int64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
  };
  std::vector<Agg> agg;
  hipEvent_t get();
};

}  // namespace stmg

struct stmg_handle {
  stmg_options opt{};
  hipStream_t stream = nullptr;
  bool stream_ordered = false;   // allocations via hipMallocAsync on `stream`
  int32_t pt = 1, q = 2, Nt = 1;
  double T = 1.0;
  std::vector<stmg::SpaceLevel> space;
  std::vector<stmg::MeshData> meshes;   // one per mesh used by some level
  std::vector<int32_t> mesh_slot;       // problem mesh index -> meshes[] slot (-1 unused)
  std::vector<stmg::LevelData> levels;
  std::vector<stmg::DevBuf> bufs;
  int64_t device_bytes = 0, factor_bytes = 0;
  double *d_partial = nullptr, *d_scalar = nullptr;
  double *d_halo = nullptr;  // residual segment hand-over, 2 * n_e (finest) values
  int32_t n_partial = 0;
  double *d_tmp[3] = {nullptr, nullptr, nullptr};
  float *f_tmp[3] = {nullptr, nullptr, nullptr};
  double bnorm = 0.0;
  std::vector<double> history;
  double setup_s = 0.0, solve_s = 0.0;
  rocblas_handle rb = nullptr;          // during the device setup phase only
  bool device_factor_on = false;        // numeric factorisation on the GPU (from device_factor)
  bool rows_hilbert = true;             // residual rows in Hilbert order (else Morton), fixed at setup
  stmg::ProfState prof_state;
  stmg::Profiler prof;
  int32_t cycles = 0;
  double rel_res = 0.0;
  // one iteration captured as a HIP graph (option graph), replayed by
  // stmg_cycles and stmg_solve; its squared residual norm lands in
  // d_scalar[GRAPH_NORM_SLOT]
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t graph_stream = nullptr;   // the capture stream
  int device = -1;                      // HIP device current at setup
  int32_t factor_workers = 1;           // threads (each with its own stream) of the slab factorisations
  std::mutex alloc_mu;                  // guards bufs, device_bytes and factor_bytes during setup
  double *noalloc_scratch = nullptr;    // that device's copy of the no-allocation scratch array
};

namespace stmg {
namespace internal {
// Phases of stmg_setup and one solver iteration, for the request server.
// All throw StmgError on failure.
stmg_handle *setup_host(const stmg_problem *prob, const stmg_options *opt);  // no HIP calls
int64_t estimate_bytes(const stmg_handle *h);                                // device bytes the next phase needs
void setup_device(stmg_handle *h, hipStream_t stream);                       // uploads on `stream`
void iteration(stmg_handle *h, double *dst_norm2);                          // enqueue one iteration on h->stream
// Handles the server batches (the same cycle shape and similar work per
// iteration), and one batched iteration on stream s (each member's squared
// residual norm into its d_scalar[0]).
bool batchable(const stmg_handle *a, const stmg_handle *b);
void batched_iteration(const std::vector<stmg_handle *> &hs, hipStream_t s);
void destroy(stmg_handle *h);
const char *last_error();
}  // namespace internal
}  // namespace stmg

