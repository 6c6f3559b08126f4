// Host runtime of libmuster: context, device arena, registration jobs and the
// launch plans that turn one optimisation iteration of many jobs into a
// fixed sequence of batched kernel launches.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/muster.h"
#include "muster_internal.h"
#include "arena.h"
#include "scheduler.h"

namespace muster {

void set_error(const char* fmt, ...);

// Thrown inside the library only (Error, scheduler.h); converted to a status
// at the ABI.
[[noreturn]] void fail(muster_status st, const char* fmt, ...);

#define MUSTER_HIP(expr)                                                              \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      ::muster::fail(MUSTER_E_DEVICE, "%s failed: %s (%s:%d)", #expr,                 \
                     hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

// The context's device memory: the arena's bookkeeping (arena.h) over HIP's
// allocator.  hipMalloc allocates on the current device, which every entry
// point sets to the context's.
struct HipDev {
  static bool alloc(size_t bytes, void** p) {
    if (hipMalloc(p, bytes) == hipSuccess && *p) return true;
    (void)hipGetLastError();
    return false;
  }
  static void free(void* p) { (void)hipFree(p); }
  static void sync(int device) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != device) (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
  }
};
using Arena = BasicArena<HipDev>;

struct KernelStats {
  int64_t launches[MUSTER_K_COUNT] = {};
  double ms[MUSTER_K_COUNT] = {};
  double bytes[MUSTER_K_COUNT] = {};
};

struct Server;

// Tile choice of the window-statistics kernels (shape index into
// SIM_SHAPE_Y/X, and the z extent of a block's chunk).
struct SimTile {
  int shape = 0;
  int zc = 32;
};

// Event pair of one timed launch, resolved at the next synchronisation.
struct TimedLaunch {
  hipEvent_t a, b;
  int k;
  double bytes;
};

struct Ctx {
  int device = 0;
  Arena arena;
  hipStream_t ws = nullptr;          // work stream (capturable)
  bool poisoned = false;
  bool timing = false;
  uint32_t timing_mask = 0;  // kernel classes whose eager launches carry events
  KernelStats stats;
  // timed launches not yet resolved, and created events kept for reuse (an
  // event pair per launch would otherwise be created and destroyed each time)
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> event_pool;
  std::mutex timing_mu;
  std::mutex mu;                     // serialises API calls that use ws
  void* step_items = nullptr;        // device buffer for single-step item tables
  size_t step_items_bytes = 0;
  double* step_acc = nullptr;        // device doubles for single-step results
  void* noalloc_scratch = nullptr;   // this device's scratch array (muster_sim_noalloc)
  std::unique_ptr<Server> server;
  // tiling of the window statistics: MUSTER_TILES_* mode, the fixed choice,
  // and the autotuner's results keyed by (D, H, W, window, metric)
  int tile_mode = MUSTER_TILES_AUTOTUNE;
  SimTile fixed_tile;
  std::map<std::vector<int>, SimTile> tuned;
  std::string tune_path;             // optional on-disk cache (MUSTER_TUNE_CACHE)
  std::mutex tune_mu;
  Ctx(uint64_t budget, int device) : arena(budget, device) {}
};

// Device allocation owned through the context's arena.
struct DevMem {
  Ctx* ctx = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() { reset(); }
  void reset() {
    if (p && ctx) ctx->arena.release(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(Ctx* c, size_t n);
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// One registration job: buffers sized for its finest grid and reused, with
// the level's own stride, at coarser levels.
struct Job {
  Ctx* ctx = nullptr;
  int N = 0;
  int dims[3] = {0, 0, 0};
  muster_params p{};
  const float* images_fine = nullptr;
  const float* svf_init = nullptr;
  float* svf_out = nullptr;
  float* pairs_out = nullptr;
  bool grad_mode = false;            // autograd: phi is the caller's, Adam writes a gradient
  float* grad_out = nullptr;
  float grad_scale = 1.f;

  int level = 0;                     // current pyramid level (0 = coarsest)
  int ff = 1;                        // flow grid factor: flows on the image grid / ff
  int ldims[MUSTER_MAX_LEVELS][3];   // flow grid per level (fields)
  int idims[MUSTER_MAX_LEVELS][3];   // image grid per level
  std::vector<int> deep_slot;        // N*N -> slot of |i-j| >= 2 pairs, -1 otherwise
  std::vector<double> times;         // acquisition times (empty if not given)
  SimTile sim_tile[MUSTER_MAX_LEVELS];

  DevMem m_phi, m_m, m_v, m_us, m_deep, m_gpair, m_pp, m_coef, m_img, m_state, m_hist;
  DevMem m_phis, m_t1, m_t2;         // smoothed flow and gradient ping-pong (smoothing on)
  DevMem m_pimg, m_gimg;             // pair fields and their gradients on the image grid (ff > 1)
  DevMem m_rigid;                    // RigidState of sessions 1..N-1 (params.rigid)
  float* rigid_out = nullptr;
  DevMem m_stage, m_desc, m_flags;   // staged Exp-backward accumulation (K >= 2)
  DevMem m_det64;                    // deterministic mode: fixed-point twins (see det64_*)
  float* phi = nullptr;              // may alias the caller's field in grad_mode
  float* mbuf = nullptr;
  float* vbuf = nullptr;
  JobState* js = nullptr;
  double* hist = nullptr;
  int hist_len = 0;
  double step_seconds = 0.0;         // wall time of the iterations run so far (see muster_report)
  std::vector<float*> level_images;  // per level: [N][V_l]
  JobState* host_state = nullptr;    // pinned
  uint64_t footprint = 0;

  ~Job();
  size_t V(int l) const { return (size_t)ldims[l][0] * ldims[l][1] * ldims[l][2]; }
  size_t VI(int l) const { return (size_t)idims[l][0] * idims[l][1] * idims[l][2]; }
  size_t VIc() const { return VI(level); }
  float* fieldI(float* base, size_t idx) const { return base + idx * 3 * VIc(); }
  float sigma() const { return p.smooth_sigma / (float)(1 << (p.levels - 1 - level)); }
  bool smoothing() const { return sigma() > 0.f; }
  // the flow Exp integrates: the smoothed field when smoothing is on
  float* flow(int i) const { return field(smoothing() ? m_phis.as<float>() : phi, (size_t)i); }
  size_t Vc() const { return V(level); }
  int K() const { return p.K; }
  float* field(float* base, size_t idx) const { return base + idx * 3 * Vc(); }
  float* us_field(int dir, int slot) const;     // see runtime.cpp
  float* u_step(int dir, int s) const;          // u_s for s in 1..K (store or recompute layout)
  float* u_final(int dir) const { return u_step(dir, p.K); }
  float* pair_field(int i, int j) const;        // U[j->i] on the flow grid
  float* pair_grad(int i, int j) const;
  float* pair_img(int i, int j) const;          // U[j->i] on the image grid
  RigidState* rigid(int j) const { return m_rigid.as<RigidState>() + (j - 1); }  // j >= 1
  float* pair_grad_img(int i, int j) const;
  float* pp(int dir, int k) const { return field(m_pp.as<float>(), (size_t)dir * 2 + k); }
  bool staged() const { return p.K >= 2; }
  int tiles_fine = 0;                // point tiles of the finest grid
  float* stage(int dir, int k) const {
    return m_stage.as<float>() + ((size_t)dir * 2 + k) * tiles_fine * 3 * STAGE_CAP;
  }
  int* desc(int dir, int k) const { return m_desc.as<int>() + ((size_t)dir * 2 + k) * tiles_fine * 8; }
  int* flag(int dir, int s) const { return m_flags.as<int>() + (size_t)dir * p.K + s; }
  bool det() const { return p.deterministic != 0; }
  // 64-bit fixed-point twins of the gradient of consecutive field dir (the
  // depth-1 pair gradient, dir = 2i for f_i, 2i+1 for b_i) and of the
  // Exp-backward ping-pong field pp(dir, k); null unless deterministic
  long long* det64_pair(int dir) const {
    return det() ? m_det64.as<long long>() + (size_t)dir * 3 * Vc() : nullptr;
  }
  long long* det64_pp(int dir, int k) const {
    return det() ? m_det64.as<long long>() + ((size_t)2 * (N - 1) + (size_t)dir * 2 + k) * 3 * Vc()
                 : nullptr;
  }
  float* coef(int i, int j) const;
  const float* image(int i) const { return level_images[level] + (size_t)i * VIc(); }
};

uint64_t job_footprint(int N, const int dims[3], const muster_params& p);
void validate_params(const muster_params& p);
void validate_problem(int N, const int dims[3], const muster_params& p, const double* times);
std::unique_ptr<Job> make_job(Ctx* ctx, const muster_job& j);
void job_begin_level(Job& job, int level, hipStream_t s);   // pyramid, init/upsample, zero state
void job_final_outputs(Job& job, hipStream_t s);           // final forward + copies to the caller
// The window-statistics tiling for one problem shape under the context's
// mode; autotuning times every candidate once on scratch data on stream s.
SimTile choose_sim_tile(Ctx* ctx, const int dims[3], int window, int metric, hipStream_t s);
void load_tune_cache(Ctx* ctx);

// A launch plan: one iteration (or a forward pass) of a set of jobs.
enum StageKind {
  ST_EXP_FWD, ST_COMPOSE_FWD, ST_SIM_STATS, ST_SIM_GRAD, ST_COMPOSE_BWD, ST_EXP_BWD, ST_ADAM,
  ST_FINISH, ST_SMOOTH, ST_UPSAMPLE, ST_UPSAMPLE_ADJ, ST_RIGID_GRAD, ST_RIGID_STEP, ST_WARP,
  ST_UNSTAGE, ST_PULL_COMBINE, ST_COMPOSE_BWD_DETMAX, ST_EXP_BWD_DETMAX, ST_DET_FOLD,
  ST_DET_CLEAR
};

struct Stage {
  StageKind kind;
  size_t off;        // byte offset of the item table in the blob
  int n_items;
  int n_tiles;
  int window = 0, metric = 0, zc = 32;
  int staged = 0;    // Exp-backward staging mode
  int reg = 0;       // Exp backward: some item adds regulariser terms
  int lds = 0;       // dynamic LDS floats (smoothing)
  int shape = 0;     // window-statistics tile shape
  double bytes = 0;  // algorithmic bytes of the launch
};

struct Plan {
  std::vector<unsigned char> blob;
  std::vector<Stage> stages;
  DevMem dev;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~Plan();
  void upload(Ctx* ctx, hipStream_t s);
  void run(Ctx* ctx, hipStream_t s);            // eager
  void capture(Ctx* ctx, hipStream_t s);
  void replay(hipStream_t s);
};

enum PlanScope { PLAN_ITERATION, PLAN_FORWARD, PLAN_LOSS_FWD, PLAN_LOSS_BWD };
std::unique_ptr<Plan> build_plan(const std::vector<Job*>& jobs, PlanScope scope);

// Serving: continuous batching over the context's work stream.  The
// scheduling (queue, admission, ticks, retirement) is the Scheduler's; the
// server owns its thread and the executor that runs the jobs with HIP.
struct Server {
  Ctx* ctx;
  std::unique_ptr<Executor> ex;
  std::unique_ptr<Scheduler> sched;
  std::thread th;
  Server(Ctx* c, int max_queue);
  ~Server();
  void loop();
};

double now_seconds();

}  // namespace muster
