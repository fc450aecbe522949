// runtime.h -- host runtime of liba2a: context, resident fields, batched solver, engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/a2a.h"
#include "a2a_kernels.h"

namespace a2a {

struct Ctx;

// status carrying the ABI error code and a message
struct Err {
  int code = A2A_OK;
};

#define A2A_HIP(ctx, call)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return (ctx)->fail(A2A_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define A2A_TRY(expr)        \
  do {                       \
    int rc_ = (expr);        \
    if (rc_ != A2A_OK) return rc_; \
  } while (0)

// ---- resident fields --------------------------------------------------------------------
struct GaugeField {
  int handle = 0;
  a2a_geom geom{};
  Geo g{};
  double* canon = nullptr;        // canonical FP64 links on the device
  void* U[4][2] = {};              // [precision][parity], built on first use
  void* HL[4][2] = {};             // [precision][parity] per-site hop links (16-bit precisions)
};

struct KappaOp {
  double kappa = 0;
  double* A64[2] = {};
  double* Ai64[2] = {};
  void* Alo[4][2] = {};
  void* Ailo[4][2] = {};
  void* AF[4][2] = {};   // full 6x6 clover blocks (16-bit precisions, matrix-core stencil)
  void* AIF[4][2] = {};
  int refs = 0;
  unsigned long long last_use = 0;
};

struct CloverField {
  int handle = 0;
  int gauge = 0;
  double csw = 0;
  double* G[2] = {};
  std::vector<std::unique_ptr<KappaOp>> kops;
};

// ---- batched solver -----------------------------------------------------------------------
struct OpEntry {
  int clover_h;
  double kappa;
  KappaOp* kop;
  OpDev dev;
  int nblk;
};

enum SlotState { SS_NEW = 0, SS_RUN, SS_DONE, SS_FAIL };
enum SolverKind { SOLVER_BICGSTAB = A2A_SOLVER_BICGSTAB, SOLVER_CGNR = A2A_SOLVER_CGNR };

struct Slot {
  int sid = -1;
  int op = -1;  // index into Solver::ops
  const double* src = nullptr;
  double* sol = nullptr;
  const double* x0 = nullptr;
  char* lo = nullptr;  // inner vectors (this slot's lane within an interleaved group, or its own arena)
  char* hi = nullptr;
  size_t lo_stride = 0, hi_stride = 0;
  long long lss = 16, lcs = 0, lss_x = 16, lxoff = 0;  // inner layout strides (SlotDev)
  char* lo_alloc = nullptr;  // allocation this slot owns (its arena, or its group's for lane 0)
  char* il_base = nullptr;   // interleaved group: arena base (group identity), tiles, lane
  int il_nt = 0, il_lane = -1;
  double tol = 1e-10, target = 0, eta_norm = 0, last_r64 = INFINITY;
  int max_iter = 10000;
  int iters = 0, rus = 0, restarts = 0, stagn = 0;
  int state = SS_NEW;
  int err = A2A_OK;
  double t_submit = 0, t_done = 0;
  a2a_solve_info info{};
  long long req = -1;
  int req_idx = 0;
};

// Launch configuration of one workload, chosen by the autotuner per (arch, lattice, inner
// precision, RHS bucket).  Zero fields mean "the context's default".
struct TuneCfg {
  int il_width = 0;           // RHS per interleaved group (16, 32 or 48 lanes; FP16 / BF16 storage)
  int by = 0, bz = 0, bt = 0;  // stencil brick extents in y, z, t (the x extent is the whole row)
  int R = 0;                  // RHS per thread of the per-thread stencil (1, 2 or 4)
  int R64 = 0;                // RHS per thread of the FP64 stencils of reliable updates (1 or 2)
  int slab = -1;              // matrix-core blocks in XCD slabs (1) or in brick order (0); -1: the option
  int by64 = 0, bz64 = 0, bt64 = 0;  // brick of the FP64 stencils (0: the operators' brick)
  int xcd64 = -1;             // FP64 stencil tiles in XCD slabs (1) or not (0); -1: the option
};

struct Solver {
  Ctx* ctx;
  int prec;
  int R;    // RHS per thread in the stencil
  int R64;  // RHS per thread in the FP64 stencils of setup, reliable updates and reconstruction
  int method = SOLVER_BICGSTAB;  // inner Krylov method of every slot of this solver
  int by = 0, bz = 0, bt = 0;    // brick of the operators this solver creates (0: the lattice's default)
  int mfma_slab = 0;             // matrix-core stencil blocks ordered in XCD slabs
  bool il_nt3 = false;           // every interleaved group has three lane tiles
  int by64 = 0, bz64 = 0, bt64 = 0;  // brick of the FP64 stencils (reliable updates; 0: the operators')
  size_t peak_live = 0;          // most slots live at once (tail checks)
  int xcd_hop = -1;              // per-thread stencil tiles of full launches in XCD slabs (1/0; -1: the option)
  int xcd_sub = -1;              // the same for subset launches (FP64 setup, reliable updates, reconstruction)
  std::vector<OpEntry> ops;
  std::vector<Slot*> live;  // slots in the device tables (running)
  // device tables
  OpDev* d_ops = nullptr;
  SlotDev* d_slots = nullptr;
  int* d_groups = nullptr;
  int2* d_hop_tiles = nullptr;
  int2* d_vec_tiles = nullptr;
  int* d_sub_groups = nullptr;
  int2* d_sub_tiles = nullptr;
  int* d_sub_list = nullptr;
  int2* d_vec_nonil = nullptr;  // per-slot tiles of the slots not in interleaved groups
  int* d_il_slots = nullptr;    // interleaved lane tiles: 16 slot indices each
  int2* d_il_tiles = nullptr;   // {lane tile, site block}
  int* d_sub_il_slots = nullptr;
  ILGroupDev* d_ilgroups = nullptr;  // interleaved groups of live slots (matrix-core stencil)
  int2* d_il_hop_tiles = nullptr;    // {group, site block}
  int* d_groups_nonil = nullptr;     // R-groups of the slots outside interleaved groups
  int2* d_hop_nonil = nullptr;
  size_t cap_ops = 0, cap_slots = 0, cap_groups = 0, cap_hop = 0, cap_vec = 0, cap_subg = 0, cap_subt = 0,
         cap_subl = 0, cap_nonil = 0, cap_ils = 0, cap_ilt = 0, cap_subils = 0, cap_ilg = 0, cap_ilh = 0,
         cap_gnonil = 0, cap_hnonil = 0;
  int n_hop_tiles = 0, n_vec_tiles = 0, n_vec_nonil = 0, n_il_tiles = 0;
  int n_il_hop_tiles = 0, n_hop_nonil = 0;
  bool il_mfma = false;  // every interleaved group's operator has its matrix-core fields
  // tile and slot counts of the last uploaded subset; its tile buffer holds
  // [hop tiles | per-slot tiles | per-slot tiles of non-interleaved slots | interleaved tiles]
  int sub_nh = 0, sub_nv = 0, sub_n = 0, sub_nn = 0, sub_ni = 0;
  bool dirty = true;
  bool with_hi = true;

  Solver(Ctx* c, int p, int r);
  ~Solver();
  int op_index(int clover_h, double kappa, KappaOp* kop, const GaugeField* gf);
  int add_slot(Slot* s);
  void gc_ops();
  int rebuild();
  // subset helpers (indices into live)
  int upload_subset(const std::vector<int>& idx, int R_sub);
  // the subset's per-slot vector tiles only (they do not depend on the group width): a no-op when
  // the last subset upload was this subset
  int upload_subset_vec(const std::vector<int>& idx);
  // the last subset upload (slot indices, group width, table generation); gen counts rebuilds
  std::vector<int> sub_idx;
  int sub_R = 0;
  unsigned sub_gen = 0, gen = 0;
  // host buffers of upload_subset's lists, kept between calls
  std::vector<int> sc_groups, sc_ils;
  std::vector<int2> sc_h, sc_v, sc_n, sc_i, sc_all;
  int finalize_red(bool sub, int kind);
  // kernel sequences
  int hop(bool sub, int n_tiles, int Rk, int psel, int kprec, int out_par, int vin, int vout, int vaux1, int vaux2,
          int vrhat, double ca, double cb, double gsign, int gpow, int inv, int red, const char* cls,
          int fin = -1,    // fin: finalize kind of the reduction (default: red itself)
          int lo_mask = 0);  // FP64 correction-form stencils: inputs from the inner arena
  int vec(bool sub, int n_tiles, int kind, int par = 0, int use_inv = 0, int vin = -1, int vout = -1);
  int layout_in(bool sub, int n_tiles, int which_in, int psel, int kprec, int ve, int vo, int g5, int red);
  int layout_out(bool sub, int n_tiles, int psel, int kprec, int ve, int vo, int g5);
  int iteration();
  int cg_direction();
  int run_steps(int iters);
  int init_kind() const { return method == SOLVER_CGNR ? VK_CG_INIT : VK_INIT; }
  int setup(const std::vector<int>& idx);
  int finish(const std::vector<int>& fin);
  int check();
  int true_residual(const std::vector<int>& idx);
  int true_residual_corr(const std::vector<int>& idx);
  // BiCGStab iterates the symmetric Schur form 1 - kappa^2 A_oo^{-1} H_oe A_ee^{-1} H_eo
  bool sym() const;
  int finalize(const std::vector<int>& idx);
  int run_until_done(int max_outer_iters);
  int retire();
};

// ---- context ------------------------------------------------------------------------------
struct EventRec {
  int cls;
  hipEvent_t a, b;
  double bytes;
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0, used = 0;
  std::unordered_map<void*, size_t> sizes;  // live allocations
  // freed blocks kept for reuse, by size: per-request slot buffers come and go with every
  // request, and hipMalloc / hipFree of hundreds of MB (hipFree waits for the device) cost
  // more than the solves of small requests.  All work on library memory is ordered on
  // `stream`, so a block can be handed out again while kernels that used it are still queued.
  // The budget limits live bytes; the cache is released when live + cached + new would exceed
  // it or hipMalloc fails.
  std::multimap<size_t, void*> cache;
  size_t cached = 0;
  std::string err;
  int next_handle = 1;
  std::map<int, std::unique_ptr<GaugeField>> gauges;
  std::map<int, std::unique_ptr<CloverField>> clovers;
  unsigned long long use_clock = 0;
  // options
  int rhs_block = 4;
  int rhs_block64 = 2;  // RHS per thread of the FP64 stencils (1 or 2)
  int check_every = 4;
  // reliable-update trigger: the iterated residual has dropped by this factor since the last
  // FP64 residual (FP16 and FP32 storage; BF16's 8-bit mantissa holds about two digits)
  double delta_lo = 0.03, delta_bf16 = 0.05, delta_64 = 1e-3;
  double delta_cgnr = 0.1;  // CGNR with FP16 storage
  int xcd_order = 1;
  int timing = 0;
  int debug = 0;  // A2A_DEBUG=1 in the environment: residual trace on stderr
  int autotune = 0;                  // pick the stencil RHS-block width per workload
  int interleave = 1;                // FP16/BF16 inner vectors in the interleaved group layout
  int mfma = 1;                      // interleaved groups use the matrix-core stencil
  int solver = SOLVER_BICGSTAB;      // inner Krylov method of solves and engine requests
  int cgnr_fallback = 1;             // BiCGStab breakdowns are finished by CGNR (solve calls)
  int force_breakdown = 0;           // test hook: BiCGStab slots break down at their first update
  bool poison = false;               // test hook: allocations are filled with 0xFF bytes (NaN)
  int fail_setup_enomem = 0;         // test hook: the next n source preparations fail (A2A_ENOMEM)
  int fail_setup_device = 0;         // test hook: the next n source preparations fail (A2A_EDEVICE)
  int il_width = IL_LANES;           // RHS per interleaved group (16, 32 or 48)
  int brick_by = 0, brick_bz = 0, brick_bt = 0;  // option "brick": stencil brick of new solvers (0: default)
  int mfma_slab = 0;                 // option "mfma_slab": matrix-core blocks in XCD slabs
  int ru_correction = 1;             // option "ru_correction": reliable updates as r64 -= M (sigma x_lo)
  double target_frac = 0.8;          // option "target_frac": Schur-residual target / (tol ||eta||)
  int tail_checks = 1;               // option "tail_checks": check every iteration in a batch's tail
  int schur_sym = 1;                 // option "schur_sym": BiCGStab on the symmetric Schur form
  std::map<std::string, TuneCfg> tuned;  // tune key -> launch configuration
  std::string tune_path;             // A2A_TUNE_CACHE: JSON file of tuned configurations
  // reduction scratch
  double* scal_pool = nullptr;
  double* scal_host = nullptr;
  // pinned staging of host-to-device table uploads (device tile lists, slot and operator
  // tables): uploads are copied here and queued without waiting; space is reused only after the
  // next stream synchronisation (sync() resets stage_off), when every queued copy has completed
  char* stage = nullptr;
  size_t stage_cap = 0, stage_off = 0;
  bool stage_failed = false;
  size_t stage_req = 0;  // option "upload_stage_bytes": staging size (0: 64 MiB)
  double* partials = nullptr;
  int partial_slots = 0, partial_blk = 0;
  std::vector<int> sid_free;
  int sid_cap = 0;
  int sid_max = -1;
  std::vector<char> sid_used;
  // kernel timing
  std::vector<EventRec> pending;
  std::vector<hipEvent_t> ev_pool;
  // timed classes: 0 schur1, 1 schur2, 2 x/r update, 3 p update, 4 s update
  static constexpr int NCLS = 5;
  long long t_launches[NCLS] = {};
  double t_ms[NCLS] = {};
  double t_bytes[NCLS] = {};  // algorithmic bytes of the timed launches

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  int dalloc(void** p, size_t n);
  void dfree(void* p);
  void release_cache();
  int alloc_sid(int nblk, int* sid);
  void free_sid(int sid);
  int ensure_partials(int nslots, int nblk);
  RedBuf redbuf() const {
    RedBuf r;
    r.partials = partials;
    r.maxblk = partial_blk;
    return r;
  }
  int sync() {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(A2A_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    stage_off = 0;  // every copy out of the staging buffer has completed
    return A2A_OK;
  }
  int read_scal() {  // whole used range of the scalar pool into host memory
    if (sid_max < 0) return A2A_OK;
    A2A_HIP(this, hipMemcpyAsync(scal_host, scal_pool, sizeof(double) * NSCAL * (sid_max + 1),
                                 hipMemcpyDeviceToHost, stream));
    return sync();
  }
  // resident fields
  GaugeField* gauge(int h) {
    auto it = gauges.find(h);
    return it == gauges.end() ? nullptr : it->second.get();
  }
  CloverField* clover(int h) {
    auto it = clovers.find(h);
    return it == clovers.end() ? nullptr : it->second.get();
  }
  int gauge_links(GaugeField* gf, int prec, void** out0, void** out1);
  int hop_links(GaugeField* gf, int prec);               // gf->HL[prec][*]
  int clover_full(KappaOp* k, int prec, long hv);        // k->AF / k->AIF [prec][*]
  int kappa_op(CloverField* cf, double kappa, int prec, KappaOp** out);
  size_t evict_unused_kops();
  int timing_begin(int cls, hipEvent_t* a);
  int timing_end(int cls, hipEvent_t a, double alg_bytes);
  int timing_collect();
};

double now_seconds();
int geom_to_geo(const a2a_geom* geom, Geo* g);
// valid stencil bricks (by, bz, bt) of a lattice in order of preference (the first is the
// default of geom_to_geo); returns how many were written (at most maxn)
int brick_choices(const Geo& g, int (*out)[3], int maxn);
void xcd_order(std::vector<int2>& tiles, bool enable);

}  // namespace a2a
