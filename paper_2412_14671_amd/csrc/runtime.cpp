// Host runtime of libmuster: context and arena, registration jobs, launch
// plans (one optimisation iteration of many jobs as a fixed sequence of
// batched launches, replayed eagerly or from a captured hipGraph), the
// continuous-batching server, and the C ABI of include/muster.h.
#include "runtime.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <tuple>

namespace muster {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

void fail(muster_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw Error{st, std::string(buf)};
}

// A named range on the profiler's marker timeline (rocprofv3
// --marker-trace): pyramid levels, the final forward pass, server ticks and
// admissions.  Without a profiler attached the calls return at once.
struct Range {
  explicit Range(const char* fmt, ...) {
    char buf[160];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    roctxRangePushA(buf);
  }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

double now_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

template <class F>
static muster_status guard(Ctx* ctx, F&& f) {
  try {
    if (ctx && ctx->poisoned) fail(MUSTER_E_DEVICE, "context poisoned by an earlier device error");
    if (ctx) MUSTER_HIP(hipSetDevice(ctx->device));
    f();
    g_err.clear();
    return MUSTER_OK;
  } catch (const Error& e) {
    g_err = e.msg;
    if (e.st == MUSTER_E_DEVICE && ctx) ctx->poisoned = true;
    return e.st;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return MUSTER_E_NOMEM;
  } catch (...) {
    g_err = "unexpected internal exception";
    return MUSTER_E_INTERNAL;
  }
}

// ---------------------------------------------------------------------------
// arena
// ---------------------------------------------------------------------------
void DevMem::alloc(Ctx* c, size_t n) {
  reset();
  ctx = c;
  p = c->arena.try_alloc(n);
  if (!p)
    fail(MUSTER_E_NOMEM, "device allocation of %zu bytes failed (arena %llu of %llu bytes in use)",
         n, (unsigned long long)c->arena.used(), (unsigned long long)c->arena.budget());
  bytes = n;
}

// ---------------------------------------------------------------------------
// validation and footprint
// ---------------------------------------------------------------------------
static int pair_index(int i, int j, int N) { return i * (N - 1) + (j < i ? j : j - 1); }

void validate_params(const muster_params& p) {
  if (p.levels < 1 || p.levels > MUSTER_MAX_LEVELS)
    fail(MUSTER_E_INVALID, "levels must be in 1..%d (got %d)", MUSTER_MAX_LEVELS, p.levels);
  for (int l = 0; l < p.levels; ++l)
    if (p.iters[l] < 0 || p.iters[l] > 1000000)
      fail(MUSTER_E_INVALID, "iters[%d] = %d out of range", l, p.iters[l]);
  if (p.K < 1 || p.K > 20) fail(MUSTER_E_INVALID, "K must be in 1..20 (got %d)", p.K);
  if (p.window != 3 && p.window != 5 && p.window != 7)
    fail(MUSTER_E_INVALID, "window must be 3, 5 or 7 (got %d)", p.window);
  if (p.metric != MUSTER_METRIC_LNCC && p.metric != MUSTER_METRIC_SILNCC)
    fail(MUSTER_E_INVALID, "unknown metric %d", p.metric);
  if (!(p.alpha_ss >= 0.f) || !std::isfinite(p.alpha_ss)) fail(MUSTER_E_INVALID, "alpha_ss must be >= 0");
  if (!(p.lr >= 0.f) || !std::isfinite(p.lr)) fail(MUSTER_E_INVALID, "lr must be >= 0");
  if (!(p.warmup >= 0.f && p.warmup <= 1.f)) fail(MUSTER_E_INVALID, "warmup must be in [0, 1]");
  if (!(p.beta1 >= 0.f && p.beta1 < 1.f) || !(p.beta2 >= 0.f && p.beta2 < 1.f) || !(p.eps > 0.f))
    fail(MUSTER_E_INVALID, "bad Adam constants");
  if (p.exp_mode != MUSTER_EXP_STORE && p.exp_mode != MUSTER_EXP_RECOMPUTE)
    fail(MUSTER_E_INVALID, "unknown exp_mode %d", p.exp_mode);
  if (!(p.smooth_sigma >= 0.f) || !(p.smooth_sigma <= MAX_SMOOTH_SIGMA))
    fail(MUSTER_E_INVALID, "smooth_sigma must be in [0, %g] (got %g)", (double)MAX_SMOOTH_SIGMA,
         (double)p.smooth_sigma);
  if (p.flow_factor != 0 && p.flow_factor != 1 && p.flow_factor != 2)
    fail(MUSTER_E_INVALID, "flow_factor must be 1 or 2 (got %d)", p.flow_factor);
  if (!(p.alpha_l2 >= 0.f) || !std::isfinite(p.alpha_l2)) fail(MUSTER_E_INVALID, "alpha_l2 must be >= 0");
  if (!(p.alpha_ts >= 0.f) || !std::isfinite(p.alpha_ts)) fail(MUSTER_E_INVALID, "alpha_ts must be >= 0");
  if (p.deterministic != 0 && p.deterministic != 1)
    fail(MUSTER_E_INVALID, "deterministic must be 0 or 1 (got %d)", p.deterministic);
}

void validate_problem(int N, const int dims[3], const muster_params& p, const double* times) {
  if (N < 2) fail(MUSTER_E_INVALID, "need at least 2 sessions (got %d)", N);
  if (N > 64) fail(MUSTER_E_INVALID, "at most 64 sessions are supported (got %d)", N);
  if (!dims) fail(MUSTER_E_INVALID, "dims is NULL");
  validate_params(p);
  const int f = 1 << (p.levels - 1);
  uint64_t V = 1;
  const int ff = p.flow_factor == 2 ? 2 : 1;
  for (int d = 0; d < 3; ++d) {
    if (dims[d] % (f * ff) != 0)
      fail(MUSTER_E_INVALID, "dims[%d] = %d is not divisible by 2^(levels-1) * flow_factor = %d",
           d, dims[d], f * ff);
    if (dims[d] / (f * ff) < 2)
      fail(MUSTER_E_INVALID, "dims[%d] = %d leaves fewer than 2 flow-grid points at the coarsest level",
           d, dims[d]);
    if (dims[d] / f < p.window)
      fail(MUSTER_E_INVALID, "dims[%d] = %d is smaller than the window at the coarsest level", d,
           dims[d]);
    if (p.smooth_sigma > 0.f && dims[d] > SMOOTH_MAX_DIM)
      fail(MUSTER_E_INVALID, "dims[%d] = %d exceeds %d, the longest line smoothing supports", d,
           dims[d], SMOOTH_MAX_DIM);
    V *= (uint64_t)dims[d];
  }
  if (V * 3 >= (uint64_t)INT32_MAX) fail(MUSTER_E_INVALID, "volume too large (%llu voxels)",
                                         (unsigned long long)V);
  if (p.smooth_sigma > 0.f) {
    // the filter's taps at every level's flow grid must fit the kernel
    for (int l = 0; l < p.levels; ++l) {
      const int lf = 1 << (p.levels - 1 - l);
      const float sg = p.smooth_sigma / (float)lf;
      for (int d = 0; d < 3; ++d) {
        const int n = dims[d] / (lf * ff);
        const int r = smooth_radius(n, sg);
        if (r > MAX_SMOOTH_RADIUS)
          fail(MUSTER_E_INVALID, "smoothing width %g at level %d needs a kernel radius of %d on a "
               "line of %d flow voxels (at most %d)", (double)sg, l, r, n, MAX_SMOOTH_RADIUS);
      }
    }
  }
  if (times) {
    for (int i = 0; i < N; ++i) {
      if (!std::isfinite(times[i])) fail(MUSTER_E_INVALID, "times[%d] is not finite", i);
      if (i > 0 && !(times[i] > times[i - 1]))
        fail(MUSTER_E_INVALID, "times must be strictly increasing (times[%d] <= times[%d])", i,
             i - 1);
    }
  }
}

static int per_dir_fields(const muster_params& p) {
  return p.exp_mode == MUSTER_EXP_STORE ? p.K : 3;
}

uint64_t job_footprint(int N, const int dims[3], const muster_params& p) {
  const int ff = p.flow_factor == 2 ? 2 : 1;
  const int fd[3] = {dims[0] / ff, dims[1] / ff, dims[2] / ff};
  const uint64_t VI = (uint64_t)dims[0] * dims[1] * dims[2];
  const uint64_t V = (uint64_t)fd[0] * fd[1] * fd[2];
  const uint64_t F = 3 * V * sizeof(float), FI = 3 * VI * sizeof(float);
  const uint64_t n1 = N - 1, P = (uint64_t)N * (N - 1), Pd = (uint64_t)(N - 1) * (N - 2);
  // flow grid: phi, m, v, Exp steps, composed pairs, pair gradients, ping-pong
  uint64_t fields = 3 * n1 + 2 * n1 * per_dir_fields(p) + std::max<uint64_t>(Pd, 1) + P + 4 * n1;
  if (p.smooth_sigma > 0.f) fields += 3 * n1;
  else if (p.K >= 2) fields += n1;  // combined gradient of the staged Exp adjoint
  uint64_t bytes = fields * F;
  // image grid: window coefficients, and with a coarser flow grid the pair
  // fields and their gradients
  bytes += P * FI;
  if (ff > 1) bytes += 2 * P * FI;
  if (p.rigid) bytes += n1 * sizeof(RigidState) + 256;
  // deterministic mode: 64-bit fixed-point twins of the consecutive-field
  // gradients and of the Exp-backward ping-pong
  if (p.deterministic) bytes += 6 * n1 * 3 * V * sizeof(long long);
  if (p.K >= 2) {
    // staging slots and descriptors of the Exp backward, per direction, two steps
    const uint64_t tiles = (uint64_t)point_tiles(fd[0], fd[1], fd[2]);
    bytes += 2 * 2 * n1 * tiles * (3 * STAGE_CAP * sizeof(float) + 8 * sizeof(int));
    bytes += 2 * n1 * p.K * sizeof(int) + 2 * 256;
  }
  uint64_t imgs = 0;
  for (int l = 0; l < p.levels - 1; ++l) {
    const int f = 1 << (p.levels - 1 - l);
    imgs += (uint64_t)N * (dims[0] / f) * (dims[1] / f) * (dims[2] / f) * sizeof(float);
  }
  uint64_t hist = 0;
  for (int l = 0; l < p.levels; ++l) hist += p.iters[l];
  bytes += imgs + hist * sizeof(double) + 4096 + 65536;
  // allocations are rounded to 256 bytes
  return bytes + 16 * 256;
}

// ---------------------------------------------------------------------------
// jobs
// ---------------------------------------------------------------------------
Job::~Job() {
  if (host_state) (void)hipHostFree(host_state);
}

float* Job::us_field(int dir, int slot) const {
  return field(m_us.as<float>(), (size_t)dir * per_dir_fields(p) + slot);
}

float* Job::u_step(int dir, int s) const {
  if (p.exp_mode == MUSTER_EXP_STORE) return us_field(dir, s - 1);
  if (s == p.K) return us_field(dir, 0);
  return us_field(dir, 1 + ((s - 1) % 2));
}

float* Job::pair_field(int i, int j) const {
  if (j == i + 1) return u_final(2 * i);
  if (j == i - 1) return u_final(2 * (i - 1) + 1);
  return field(m_deep.as<float>(), (size_t)deep_slot[i * N + j]);
}

float* Job::pair_grad(int i, int j) const {
  return field(m_gpair.as<float>(), (size_t)pair_index(i, j, N));
}

float* Job::coef(int i, int j) const {
  return fieldI(m_coef.as<float>(), (size_t)pair_index(i, j, N));
}

float* Job::pair_img(int i, int j) const {
  if (ff == 1) return pair_field(i, j);
  return fieldI(m_pimg.as<float>(), (size_t)pair_index(i, j, N));
}

float* Job::pair_grad_img(int i, int j) const {
  if (ff == 1) return pair_grad(i, j);
  return fieldI(m_gimg.as<float>(), (size_t)pair_index(i, j, N));
}

std::unique_ptr<Job> make_job(Ctx* ctx, const muster_job& jd) {
  validate_problem(jd.N, jd.dims, jd.params, jd.times_host);
  if (!jd.images_dev) fail(MUSTER_E_INVALID, "images is NULL");
  if (jd.params.alpha_ts > 0.f && jd.N >= 3 && !jd.times_host)
    fail(MUSTER_E_INVALID, "alpha_ts > 0 needs the acquisition times");
  auto job = std::make_unique<Job>();
  Job& J = *job;
  J.ctx = ctx;
  J.N = jd.N;
  std::memcpy(J.dims, jd.dims, sizeof J.dims);
  J.p = jd.params;
  J.images_fine = jd.images_dev;
  J.svf_init = jd.svf_init_dev;
  J.svf_out = jd.svf_out_dev;
  J.pairs_out = jd.pairs_out_dev;
  if (jd.times_host) J.times.assign(jd.times_host, jd.times_host + jd.N);
  const int L = J.p.levels;
  J.ff = J.p.flow_factor == 2 ? 2 : 1;
  for (int l = 0; l < L; ++l) {
    const int f = 1 << (L - 1 - l);
    for (int d = 0; d < 3; ++d) {
      J.idims[l][d] = jd.dims[d] / f;
      J.ldims[l][d] = jd.dims[d] / (f * J.ff);
    }
  }
  const int N = J.N;
  J.deep_slot.assign((size_t)N * N, -1);
  int slot = 0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      if (std::abs(i - j) >= 2) J.deep_slot[i * N + j] = slot++;
  const size_t V0 = J.V(L - 1);
  const size_t F = 3 * V0 * sizeof(float);
  const size_t FI = 3 * J.VI(L - 1) * sizeof(float);
  const size_t n1 = N - 1;
  const size_t P = (size_t)N * (N - 1);
  J.m_phi.alloc(ctx, n1 * F);
  J.m_m.alloc(ctx, n1 * F);
  J.m_v.alloc(ctx, n1 * F);
  J.m_us.alloc(ctx, 2 * n1 * per_dir_fields(J.p) * F);
  J.m_deep.alloc(ctx, std::max<size_t>(slot, 1) * F);
  J.m_gpair.alloc(ctx, P * F);
  J.m_pp.alloc(ctx, 4 * n1 * F);
  J.m_coef.alloc(ctx, P * FI);
  if (J.ff > 1) {
    J.m_pimg.alloc(ctx, P * FI);
    J.m_gimg.alloc(ctx, P * FI);
  }
  if (J.p.smooth_sigma > 0.f) {
    J.m_phis.alloc(ctx, n1 * F);
    J.m_t1.alloc(ctx, n1 * F);
    J.m_t2.alloc(ctx, n1 * F);
  } else if (J.staged()) {
    J.m_t1.alloc(ctx, n1 * F);  // the combined SVF gradient Adam reads
  }
  J.tiles_fine = point_tiles(J.ldims[L - 1][0], J.ldims[L - 1][1], J.ldims[L - 1][2]);
  J.rigid_out = jd.rigid_out_dev;
  if (J.p.rigid) {
    J.m_rigid.alloc(ctx, n1 * sizeof(RigidState));
    std::vector<RigidState> z(n1);
    std::memset(z.data(), 0, n1 * sizeof(RigidState));
    MUSTER_HIP(hipMemcpy(J.m_rigid.p, z.data(), n1 * sizeof(RigidState), hipMemcpyHostToDevice));
  }
  if (J.p.deterministic) {
    J.m_det64.alloc(ctx, 6 * n1 * 3 * V0 * sizeof(long long));
    // zero bits: the fixed-point fields start (and are left by every fold) at 0
    MUSTER_HIP(launch_fill(J.m_det64.as<float>(), (int64_t)(12 * n1 * 3 * V0), 0.f, nullptr));
    MUSTER_HIP(hipStreamSynchronize(nullptr));
  }
  if (J.staged()) {
    J.m_stage.alloc(ctx, 2 * 2 * n1 * (size_t)J.tiles_fine * 3 * STAGE_CAP * sizeof(float));
    J.m_desc.alloc(ctx, 2 * 2 * n1 * (size_t)J.tiles_fine * 8 * sizeof(int));
    J.m_flags.alloc(ctx, 2 * n1 * (size_t)J.p.K * sizeof(int));
  }
  size_t img = 0;
  for (int l = 0; l < L - 1; ++l) img += (size_t)N * J.VI(l);
  J.m_img.alloc(ctx, std::max<size_t>(img, 1) * sizeof(float));
  J.m_state.alloc(ctx, sizeof(JobState));
  J.hist_len = 0;
  for (int l = 0; l < L; ++l) J.hist_len += J.p.iters[l];
  J.m_hist.alloc(ctx, std::max(J.hist_len, 1) * sizeof(double));
  J.phi = J.m_phi.as<float>();
  J.mbuf = J.m_m.as<float>();
  J.vbuf = J.m_v.as<float>();
  J.js = J.m_state.as<JobState>();
  J.hist = J.m_hist.as<double>();
  J.level_images.resize(L);
  size_t off = 0;
  for (int l = 0; l < L - 1; ++l) {
    J.level_images[l] = J.m_img.as<float>() + off;
    off += (size_t)N * J.VI(l);
  }
  J.level_images[L - 1] = const_cast<float*>(J.images_fine);
  MUSTER_HIP(hipHostMalloc((void**)&J.host_state, sizeof(JobState), hipHostMallocDefault));
  std::memset(J.host_state, 0, sizeof(JobState));
  J.footprint = J.m_phi.bytes + J.m_m.bytes + J.m_v.bytes + J.m_us.bytes + J.m_deep.bytes +
                J.m_gpair.bytes + J.m_pp.bytes + J.m_coef.bytes + J.m_img.bytes +
                J.m_state.bytes + J.m_hist.bytes + J.m_phis.bytes + J.m_t1.bytes + J.m_t2.bytes +
                J.m_stage.bytes + J.m_desc.bytes + J.m_flags.bytes + J.m_pimg.bytes +
                J.m_gimg.bytes + J.m_rigid.bytes + J.m_det64.bytes;
  return job;
}

// Small item tables used outside plans (pyramid, upsampling) go through this
// helper: upload, launch, synchronise.
template <class Item, class Launch>
static void run_items(Ctx* ctx, std::vector<Item>& items, int n_tiles, hipStream_t s,
                      Launch&& launch) {
  if (items.empty() || n_tiles <= 0) return;
  DevMem d;
  d.alloc(ctx, items.size() * sizeof(Item));
  MUSTER_HIP(hipMemcpyAsync(d.p, items.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice, s));
  MUSTER_HIP(launch(d.as<Item>(), (int)items.size(), n_tiles, s));
  MUSTER_HIP(hipStreamSynchronize(s));
}

static int elem_tiles(size_t n) { return (int)((n + ELEM_PER_BLOCK - 1) / ELEM_PER_BLOCK); }

// Rigid states at the start of a level: translations doubled when the grid
// doubles, Adam moments and sums cleared, the applied displacement
// recomputed about the level's centre.
static void rigid_begin_level(Job& J, int level, hipStream_t s) {
  const size_t n1 = J.N - 1;
  std::vector<RigidState> st(n1);
  MUSTER_HIP(hipMemcpyAsync(st.data(), J.m_rigid.p, n1 * sizeof(RigidState),
                            hipMemcpyDeviceToHost, s));
  MUSTER_HIP(hipStreamSynchronize(s));
  const int* d = J.idims[level];
  const float c[3] = {0.5f * (d[0] - 1), 0.5f * (d[1] - 1), 0.5f * (d[2] - 1)};
  for (RigidState& r : st) {
    if (level > 0)
      for (int k = 0; k < 3; ++k) r.t[k] *= 2.f;
    for (int k = 0; k < 6; ++k) r.m[k] = r.v[k] = 0.f;
    for (int k = 0; k < 3; ++k) r.gsum[k] = 0.0;
    for (int k = 0; k < 9; ++k) r.gmom[k] = 0.0;
    float R[9];
    rigid_rotation(r.theta, -1, R);
    for (int a = 0; a < 3; ++a) {
      float rc = 0.f;
      for (int b = 0; b < 3; ++b) {
        r.A[3 * a + b] = R[3 * a + b] - (a == b ? 1.f : 0.f);
        rc += R[3 * a + b] * c[b];
      }
      r.off[a] = c[a] + r.t[a] - rc;
    }
  }
  MUSTER_HIP(hipMemcpyAsync(J.m_rigid.p, st.data(), n1 * sizeof(RigidState),
                            hipMemcpyHostToDevice, s));
  MUSTER_HIP(hipStreamSynchronize(s));
}

void job_begin_level(Job& J, int level, hipStream_t s) {
  Ctx* ctx = J.ctx;
  const int L = J.p.levels;
  const int N = J.N;
  if (level == 0 && L > 1) {
    // image pyramid: repeated 2x2x2 means from the finest level down
    for (int l = L - 2; l >= 0; --l) {
      std::vector<PoolItem> items;
      int tiles = 0;
      const int* dd = J.idims[l + 1];
      const size_t Vs = J.VI(l + 1), Vd = J.VI(l);
      for (int i = 0; i < N; ++i) {
        PoolItem it{};
        it.tile0 = tiles;
        it.D = dd[0]; it.H = dd[1]; it.W = dd[2];
        it.src = J.level_images[l + 1] + (size_t)i * Vs;
        it.dst = J.level_images[l] + (size_t)i * Vd;
        items.push_back(it);
        tiles += elem_tiles(Vd);
      }
      run_items(ctx, items, tiles, s, launch_pool2);
    }
  }
  J.level = level;
  const size_t V = J.Vc();
  const size_t n1 = N - 1;
  if (!J.grad_mode) {
    if (level == 0) {
      if (J.svf_init)
        MUSTER_HIP(hipMemcpyAsync(J.phi, J.svf_init, n1 * 3 * V * sizeof(float),
                                  hipMemcpyDeviceToDevice, s));
      else
        MUSTER_HIP(launch_fill(J.phi, (int64_t)(n1 * 3 * V), 0.f, s));
    } else {
      // phi_fine(x) = 2 phi_coarse((x - 0.5)/2), into the m buffer, then swap
      std::vector<UpItem> items;
      int tiles = 0;
      const int* dc = J.ldims[level - 1];
      const size_t Vcoarse = J.V(level - 1);
      for (size_t i = 0; i < n1; ++i) {
        UpItem it{};
        it.tile0 = tiles;
        it.D = dc[0]; it.H = dc[1]; it.W = dc[2];
        it.src = J.phi + i * 3 * Vcoarse;
        it.dst = J.mbuf + i * 3 * V;
        items.push_back(it);
        tiles += up_tiles(dc[0], dc[1], dc[2]);
      }
      run_items(ctx, items, tiles, s, launch_upsample2);
      std::swap(J.phi, J.mbuf);
    }
    MUSTER_HIP(launch_fill(J.mbuf, (int64_t)(n1 * 3 * V), 0.f, s));
    MUSTER_HIP(launch_fill(J.vbuf, (int64_t)(n1 * 3 * V), 0.f, s));
  }
  MUSTER_HIP(launch_fill(J.m_pp.as<float>(), (int64_t)(4 * n1 * 3 * V), 0.f, s));
  if (J.p.rigid) rigid_begin_level(J, level, s);
  if (J.staged())  // the flags are ints; 0.0f has the same bits as 0
    MUSTER_HIP(launch_fill((float*)J.m_flags.p, (int64_t)(2 * n1 * J.p.K), 0.f, s));
  JobState st{};
  const int prev_nonfinite = level > 0 ? J.host_state->nonfinite : 0;
  st.t = 0;
  st.T = J.p.iters[level];
  st.W = std::max(1, (int)std::ceil((double)J.p.warmup * st.T));
  st.nonfinite = prev_nonfinite;
  st.lr0 = J.p.lr;
  st.b1 = J.p.beta1;
  st.b2 = J.p.beta2;
  st.eps = J.p.eps;
  st.history = J.hist;
  st.hist_len = J.hist_len;
  st.flags = J.staged() ? J.m_flags.as<int>() : nullptr;
  st.n_flags = J.staged() ? (int)(2 * n1 * J.p.K) : 0;
  int base = 0;
  for (int l = 0; l < level; ++l) base += J.p.iters[l];
  st.hist_base = base;
  *J.host_state = st;
  MUSTER_HIP(hipMemcpyAsync(J.js, J.host_state, sizeof(JobState), hipMemcpyHostToDevice, s));
  // a deterministic job's result must not depend on timing: it takes the
  // context's fixed tiling if one is set, else the default one
  if (J.det() && ctx->tile_mode == MUSTER_TILES_AUTOTUNE) {
    J.sim_tile[level].shape = 0;
    J.sim_tile[level].zc = std::min(32, J.idims[level][0]);
  } else {
    J.sim_tile[level] = choose_sim_tile(ctx, J.idims[level], J.p.window, J.p.metric, s);
  }
  MUSTER_HIP(hipStreamSynchronize(s));
}

static void read_state(Job& J, hipStream_t s) {
  MUSTER_HIP(hipMemcpyAsync(J.host_state, J.js, sizeof(JobState), hipMemcpyDeviceToHost, s));
  MUSTER_HIP(hipStreamSynchronize(s));
}

void job_final_outputs(Job& J, hipStream_t s) {
  Range range("muster final outputs: N %d", J.N);
  Ctx* ctx = J.ctx;
  std::vector<Job*> one{&J};
  auto plan = build_plan(one, PLAN_FORWARD);
  plan->upload(ctx, s);
  plan->run(ctx, s);
  const size_t VI = J.VIc();
  if (J.svf_out) {
    if (J.ff == 1) {
      MUSTER_HIP(hipMemcpyAsync(J.svf_out, J.flow(0), (size_t)(J.N - 1) * 3 * VI * sizeof(float),
                                hipMemcpyDeviceToDevice, s));
    } else {
      // the flows carried up to the image grid (image voxel units)
      std::vector<UpItem> items;
      int tiles = 0;
      for (int i = 0; i < J.N - 1; ++i) {
        UpItem it{};
        it.tile0 = tiles;
        it.D = J.ldims[J.level][0]; it.H = J.ldims[J.level][1]; it.W = J.ldims[J.level][2];
        it.src = J.flow(i);
        it.dst = J.svf_out + (size_t)i * 3 * VI;
        items.push_back(it);
        tiles += up_tiles(it.D, it.H, it.W);
      }
      run_items(ctx, items, tiles, s, launch_upsample2);
    }
  }
  if (J.pairs_out) {
    const int* d = J.idims[J.level];
    for (int i = 0; i < J.N; ++i)
      for (int j = 0; j < J.N; ++j) {
        if (i == j) continue;
        float* dst = J.pairs_out + (size_t)pair_index(i, j, J.N) * 3 * VI;
        MUSTER_HIP(hipMemcpyAsync(dst, J.pair_img(i, j), 3 * VI * sizeof(float),
                                  hipMemcpyDeviceToDevice, s));
        // the total deformation: the rigid part of the source session added
        if (J.p.rigid && j >= 1)
          MUSTER_HIP(launch_add_rigid(GridDims{d[0], d[1], d[2]}, dst, J.rigid(j), s));
      }
  }
  if (J.p.rigid && J.rigid_out) {
    const size_t n1 = J.N - 1;
    std::vector<RigidState> st(n1);
    MUSTER_HIP(hipMemcpyAsync(st.data(), J.m_rigid.p, n1 * sizeof(RigidState),
                              hipMemcpyDeviceToHost, s));
    MUSTER_HIP(hipStreamSynchronize(s));
    std::vector<float> out(6 * n1);
    for (size_t j = 0; j < n1; ++j)
      for (int k = 0; k < 3; ++k) {
        out[6 * j + k] = st[j].theta[k];
        out[6 * j + 3 + k] = st[j].t[k];
      }
    MUSTER_HIP(hipMemcpyAsync(J.rigid_out, out.data(), out.size() * sizeof(float),
                              hipMemcpyHostToDevice, s));
  }
  MUSTER_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
namespace {

// Algorithmic bytes per voxel (the unique bytes each step must move).
constexpr double B_EXP_FWD = 24, B_COMPOSE_FWD = 36, B_SIM_STATS = 20, B_SIM_GRAD = 32,
                 B_COMPOSE_BWD = 84, B_EXP_BWD = 60, B_ADAM = 96, B_SMOOTH = 24, B_WARP = 20,
                 B_UNSTAGE = 24;

struct Builder {
  Plan* plan;
  template <class Item>
  void add(StageKind kind, std::vector<Item>& items, int tiles, double bytes, int window = 0,
           int metric = 0, int zc = 32) {
    if (items.empty()) return;
    size_t off = (plan->blob.size() + 63) & ~(size_t)63;
    plan->blob.resize(off + items.size() * sizeof(Item));
    std::memcpy(plan->blob.data() + off, items.data(), items.size() * sizeof(Item));
    Stage st;
    st.kind = kind;
    st.off = off;
    st.n_items = (int)items.size();
    st.n_tiles = tiles;
    st.window = window;
    st.metric = metric;
    st.zc = zc;
    st.bytes = bytes;
    plan->stages.push_back(st);
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// Taps of the smoothing filter.  Appendix A filters in the Fourier domain with
// the transfer function exp(-(omega / omega_s)^2 / 2), omega_s = 1 / sigma.
// On a periodic line of n samples the filter is the circular convolution with
// h[m] = (1/n) sum_k exp(-sigma^2 omega_k^2 / 2) cos(omega_k m), where
// omega_k = 2 pi min(k, n - k) / n are the line's DFT frequencies in radians
// per sample; the 3-D transfer is the product of the three axes', so one
// pass per axis gives the whole filter.  The taps are kept out to the
// smallest radius beyond which they sum to less than 2^-26 in magnitude (well
// under float rounding of a unit-sum filter), or over the whole line when the
// spectrum is still large at Nyquist and the taps ring all the way round
// (small sigma).  The whole line of an even n is taken as offsets -n/2..n/2
// with half of h[n/2] at each end, so that the taps stay symmetric.
// ---------------------------------------------------------------------------
namespace {

struct SmoothTaps {
  int radius = 0;
  std::vector<double> w;  // offsets -radius..radius
};

const SmoothTaps& smooth_taps(int n, float sigma) {
  static std::mutex mu;
  static std::map<std::pair<int, float>, SmoothTaps> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_pair(n, sigma);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const double sg = sigma, two_pi = 2.0 * M_PI;
  std::vector<double> H(n / 2 + 1);
  for (int k = 0; k <= n / 2; ++k) {
    const double om = two_pi * k / n;
    H[k] = std::exp(-0.5 * sg * sg * om * om);
  }
  // h[m] for m = 0..n/2: the k and n-k terms of the sum are equal
  std::vector<double> h(n / 2 + 1);
  for (int m = 0; m <= n / 2; ++m) {
    double acc = H[0];
    for (int k = 1; 2 * k < n; ++k) acc += 2.0 * H[k] * std::cos(two_pi * (double)k * m / n);
    if (n % 2 == 0) acc += H[n / 2] * ((m & 1) ? -1.0 : 1.0);
    h[m] = acc / n;
  }
  // distinct offsets of the line: +-1..+-(n-1)/2, and n/2 once when n is even
  const int half = (n - 1) / 2;
  const double tol = std::ldexp(1.0, -26);
  double tail = (n % 2 == 0 && n >= 2) ? std::fabs(h[n / 2]) : 0.0;
  int r = half;
  while (r > 0 && tail + 2.0 * std::fabs(h[r]) <= tol) {
    tail += 2.0 * std::fabs(h[r]);
    --r;
  }
  SmoothTaps t;
  if (r == half && n % 2 == 0 && n >= 2 && tail > tol) {
    // the whole line of an even n
    t.radius = n / 2;
    t.w.assign(2 * t.radius + 1, 0.0);
    for (int m = -t.radius; m <= t.radius; ++m) t.w[m + t.radius] = h[std::abs(m)];
    t.w[0] *= 0.5;
    t.w[2 * t.radius] *= 0.5;
  } else {
    t.radius = r;
    t.w.assign(2 * r + 1, 0.0);
    for (int m = -r; m <= r; ++m) t.w[m + r] = h[std::abs(m)];
  }
  return cache.emplace(key, std::move(t)).first->second;
}

}  // namespace

int smooth_radius(int n, float sigma) { return smooth_taps(n, sigma).radius; }

int smooth_item_setup(SmoothItem& it, const int dims[3], int axis, float sigma, int* lds_floats) {
  it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
  it.axis = axis;
  const SmoothTaps& tp = smooth_taps(dims[axis], sigma);
  const int r = tp.radius;
  if (r > MAX_SMOOTH_RADIUS)
    fail(MUSTER_E_INVALID, "smoothing sigma %g on a line of %d voxels needs a kernel radius of %d "
         "(at most %d)", (double)sigma, dims[axis], r, MAX_SMOOTH_RADIUS);
  it.radius = r;
  for (int k = 0; k < SMOOTH_WLEN; ++k) it.w[k] = 0.f;
  for (int k = 0; k <= 2 * r; ++k) it.w[SMOOTH_WPAD + k] = (float)tp.w[k];
  // LDS floats a tile of L lines needs, and the number of lines on offer
  const int n = dims[axis];
  const int avail = axis == 2 ? dims[0] * dims[1] : dims[2];
  auto need = [&](int L) { return axis == 2 ? 2 * L * (dims[2] | 1) : n * L; };
  int L = 64;
  while (L > 1 && (L / 2 >= avail || need(L) > SMOOTH_LDS_TARGET)) L /= 2;
  while (L > 1 && need(L) > SMOOTH_LDS) L /= 2;
  it.lines = L;
  it.lshift = 0;
  while ((1 << it.lshift) < L) ++it.lshift;
  it.tiles_comp = axis == 2 ? (avail + L - 1) / L
                            : (axis == 0 ? dims[1] : dims[0]) * ((dims[2] + L - 1) / L);
  *lds_floats = std::max(*lds_floats, need(L));
  return 3 * it.tiles_comp;
}

namespace {

// One separable smoothing pass (axis) for every interval of the smoothing
// jobs: src(i) -> dst(i).
template <class SrcF, class DstF>
void add_smooth_pass(Builder& b, const std::vector<Job*>& jobs, int axis, SrcF src, DstF dst) {
  std::vector<SmoothItem> items;
  int tiles = 0, lds = 0;
  double bytes = 0;
  for (Job* J : jobs) {
    if (!J->smoothing()) continue;
    for (int i = 0; i < J->N - 1; ++i) {
      SmoothItem it{};
      it.tile0 = tiles;
      tiles += smooth_item_setup(it, J->ldims[J->level], axis, J->sigma(), &lds);
      it.src = src(J, i);
      it.dst = dst(J, i);
      items.push_back(it);
      bytes += B_SMOOTH * J->Vc();
    }
  }
  b.add(ST_SMOOTH, items, tiles, bytes);
  if (!items.empty()) b.plan->stages.back().lds = lds;
}

// phi -> smoothed flow: z into t1, y into t2, x into the flow buffer
void add_smooth_flow(Builder& b, const std::vector<Job*>& jobs) {
  auto phi = [](Job* J, int i) { return (const float*)J->field(J->phi, i); };
  auto t1 = [](Job* J, int i) { return J->field(J->m_t1.as<float>(), i); };
  auto t2 = [](Job* J, int i) { return J->field(J->m_t2.as<float>(), i); };
  auto fl = [](Job* J, int i) { return J->flow(i); };
  add_smooth_pass(b, jobs, 0, phi, t1);
  add_smooth_pass(b, jobs, 1, [&](Job* J, int i) { return (const float*)t1(J, i); }, t2);
  add_smooth_pass(b, jobs, 2, [&](Job* J, int i) { return (const float*)t2(J, i); }, fl);
}


void add_exp_fwd_step(Builder& b, const std::vector<Job*>& jobs, int s, bool recompute_only,
                      int upto) {
  // One squaring s -> s+1 for every direction of every job.  With
  // recompute_only, this is step s of recomputing u_upto in the scratch slots.
  std::vector<ExpFwdItem> items;
  int tiles = 0;
  double bytes = 0;
  for (Job* J : jobs) {
    if (s >= J->K()) continue;
    if (recompute_only && (J->p.exp_mode != MUSTER_EXP_RECOMPUTE || upto > J->K() - 1)) continue;
    const int* d = J->ldims[J->level];
    const float scale = std::ldexp(1.f, -J->K());
    for (int dir = 0; dir < 2 * (J->N - 1); ++dir) {
      const int i = dir / 2;
      const float sign = (dir % 2 == 0) ? 1.f : -1.f;
      ExpFwdItem it{};
      it.tile0 = tiles;
      it.D = d[0]; it.H = d[1]; it.W = d[2];
      if (s == 0) {
        it.src = J->flow(i);
        it.a = sign * scale;
      } else {
        it.src = J->u_step(dir, s);
        it.a = 1.f;
      }
      it.dst = J->u_step(dir, s + 1);
      items.push_back(it);
      tiles += point_tiles(d[0], d[1], d[2]);
      bytes += B_EXP_FWD * J->Vc();
    }
  }
  b.add(ST_EXP_FWD, items, tiles, bytes);
}

// Jobs whose flow grid is coarser than the image grid: the pair fields
// carried up to the image grid for the similarity (forward), or the pair
// gradients carried back down by the adjoint (backward).
constexpr double B_UPSAMPLE = 12 + 12 * 8, B_UPSAMPLE_ADJ = 12 * 8 + 12;  // per coarse voxel
void add_pair_resampling(Builder& b, const std::vector<Job*>& jobs, bool adjoint) {
  std::vector<UpItem> items;
  int tiles = 0;
  double bytes = 0;
  for (Job* J : jobs) {
    if (J->ff == 1) continue;
    const int* d = J->ldims[J->level];
    for (int i = 0; i < J->N; ++i)
      for (int j = 0; j < J->N; ++j) {
        if (i == j) continue;
        UpItem it{};
        it.tile0 = tiles;
        it.D = d[0]; it.H = d[1]; it.W = d[2];
        if (adjoint) {
          it.src = J->pair_grad_img(i, j);
          it.dst = J->pair_grad(i, j);
          tiles += up_adj_tiles(d[0], d[1], d[2]);
          bytes += B_UPSAMPLE_ADJ * J->Vc();
        } else {
          it.src = J->pair_field(i, j);
          it.dst = J->pair_img(i, j);
          tiles += up_tiles(d[0], d[1], d[2]);
          bytes += B_UPSAMPLE * J->Vc();
        }
        items.push_back(it);
      }
  }
  b.add(adjoint ? ST_UPSAMPLE_ADJ : ST_UPSAMPLE, items, tiles, bytes);
}

void add_forward(Builder& b, const std::vector<Job*>& jobs) {
  int maxK = 0, maxN = 0;
  for (Job* J : jobs) {
    maxK = std::max(maxK, J->K());
    maxN = std::max(maxN, J->N);
  }
  add_smooth_flow(b, jobs);
  for (int s = 0; s < maxK; ++s) add_exp_fwd_step(b, jobs, s, false, 0);
  for (int d = 2; d < maxN; ++d) {
    std::vector<ComposeItem> items;
    int tiles = 0;
    double bytes = 0;
    for (Job* J : jobs) {
      const int N = J->N;
      if (d >= N) continue;
      const int* dd = J->ldims[J->level];
      for (int i = 0; i < N; ++i) {
        for (int j : {i + d, i - d}) {
          if (j < 0 || j >= N) continue;
          ComposeItem it{};
          it.tile0 = tiles;
          it.D = dd[0]; it.H = dd[1]; it.W = dd[2];
          if (j > i) {
            it.prev = J->pair_field(i, j - 1);
            it.C = J->u_final(2 * (j - 1));
          } else {
            it.prev = J->pair_field(i, j + 1);
            it.C = J->u_final(2 * j + 1);
          }
          it.out = J->pair_field(i, j);
          items.push_back(it);
          tiles += point_tiles(dd[0], dd[1], dd[2]);
          bytes += B_COMPOSE_FWD * J->Vc();
        }
      }
    }
    b.add(ST_COMPOSE_FWD, items, tiles, bytes);
  }
  add_pair_resampling(b, jobs, false);
}

// Rigid adjustment (Sec. 2.5): the gradient sums of every pair whose source
// is session j >= 1 (its dSim/dU on the image grid, before the composition
// adjoints add to it), then one Adam step per session.
void add_rigid_stages(Builder& b, const std::vector<Job*>& jobs) {
  std::vector<RigidGradItem> gi;
  std::vector<RigidStepItem> si;
  int tiles = 0;
  double bytes = 0;
  for (Job* J : jobs) {
    if (!J->p.rigid) continue;
    const int* d = J->idims[J->level];
    for (int i = 0; i < J->N; ++i)
      for (int j = 1; j < J->N; ++j) {
        if (i == j) continue;
        RigidGradItem it{};
        it.tile0 = tiles;
        it.D = d[0]; it.H = d[1]; it.W = d[2];
        it.G = J->pair_grad_img(i, j);
        it.rg = J->rigid(j);
        gi.push_back(it);
        tiles += elem_tiles(J->VIc());
        bytes += 12.0 * J->VIc();
      }
    const float rmax = 0.5f * (float)(std::max(d[0], std::max(d[1], d[2])) - 1);
    for (int j = 1; j < J->N; ++j) {
      RigidStepItem it{};
      it.rg = J->rigid(j);
      it.js = J->js;
      for (int k = 0; k < 3; ++k) it.c[k] = 0.5f * (d[k] - 1);
      it.rot_lr = 1.f / rmax;
      si.push_back(it);
    }
  }
  b.add(ST_RIGID_GRAD, gi, tiles, bytes);
  b.add(ST_RIGID_STEP, si, (int)si.size(), 0.0);
}

// The pair items of the jobs whose window statistics use tile shape `shape`.
std::vector<SimItem> sim_items(const std::vector<Job*>& jobs, int shape, int& tiles, double& vox) {
  std::vector<SimItem> items;
  tiles = 0;
  vox = 0;
  for (Job* J : jobs) {
    const SimTile& tl = J->sim_tile[J->level];
    if (tl.shape != shape) continue;
    const int N = J->N;
    const int* d = J->idims[J->level];
    const int r = (J->p.window - 1) / 2;
    const double nr = (double)(d[0] - 2 * r) * (d[1] - 2 * r) * (d[2] - 2 * r);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        if (i == j) continue;
        SimItem it{};
        it.tile0 = tiles;
        it.D = d[0]; it.H = d[1]; it.W = d[2];
        it.zc = tl.zc;
        it.F = J->image(i);
        it.I = J->image(j);
        it.U = J->pair_img(i, j);
        it.coef = J->coef(i, j);
        it.gU = J->pair_grad_img(i, j);
        it.M = it.gU;  // free until k_sim_grad writes gU
        it.inv_nr = 1.0 / nr;
        it.js = J->js;
        it.sim_out = nullptr;
        it.rigid = (J->p.rigid && j >= 1) ? J->rigid(j) : nullptr;
        items.push_back(it);
        tiles += stat_tiles(d[0], d[1], d[2], tl.zc, shape);
        vox += (double)J->VIc();
      }
  }
  return items;
}

// One window-statistics stage per tile shape in use; the statistics are
// preceded by the warp of every pair's source image.
void add_sim_stages(Builder& b, const std::vector<Job*>& jobs, StageKind kind) {
  const int window = jobs[0]->p.window, metric = jobs[0]->p.metric;
  if (kind == ST_SIM_STATS) {
    std::vector<SimItem> items;
    int tiles = 0;
    double vox = 0;
    for (int shape = 0; shape < SIM_SHAPES; ++shape) {
      int t;
      double v;
      for (SimItem it : sim_items(jobs, shape, t, v)) {
        it.tile0 = tiles;
        tiles += point_tiles(it.D, it.H, it.W);
        vox += (double)it.D * it.H * it.W;
        items.push_back(it);
      }
    }
    b.add(ST_WARP, items, tiles, B_WARP * vox);
  }
  for (int shape = 0; shape < SIM_SHAPES; ++shape) {
    int tiles;
    double vox;
    auto items = sim_items(jobs, shape, tiles, vox);
    if (items.empty()) continue;
    const double per = kind == ST_SIM_STATS ? B_SIM_STATS : B_SIM_GRAD;
    b.add(kind, items, tiles, per * vox, window, kind == ST_SIM_STATS ? metric : 0);
    b.plan->stages.back().shape = shape;
  }
}

// L_L2 and L_ts terms of interval i (Sec. 2.4), on the flows Exp integrates.
// Gradient weights carry 2^K: the step-0 own term is scaled by 2^-K when the
// two directions are combined.
void set_reg_ext(ExpBwdItem& it, const Job& J, int i) {
  const int N = J.N;
  const double V = (double)J.Vc();
  const bool l2 = J.p.alpha_l2 > 0.f;
  const bool ts = J.p.alpha_ts > 0.f && N >= 3;
  if (!l2 && !ts) return;
  const double k2 = std::ldexp(1.0, J.K());
  double w_self = 0, w_prev = 0, w_next = 0;
  it.ext = 1;
  if (l2) {
    w_self += 2.0 * J.p.alpha_l2 / ((N - 1) * V);
    it.l2_loss_w = (float)(J.p.alpha_l2 / ((N - 1) * V));
  }
  if (ts) {
    const double c = 2.0 * J.p.alpha_ts / ((N - 2) * V);
    const double di = J.times[i + 1] - J.times[i];
    if (i >= 1) {
      const double dp = J.times[i] - J.times[i - 1];
      w_self += c / (di * di);
      w_prev = -c / (dp * di);
      it.flow_prev = J.flow(i - 1);
      it.ts_loss_w = (float)(J.p.alpha_ts / ((N - 2) * V));
      it.inv_dprev = (float)(1.0 / dp);
      it.inv_dself = (float)(1.0 / di);
    }
    if (i <= N - 3) {
      const double dn = J.times[i + 2] - J.times[i + 1];
      w_self += c / (di * di);
      w_next = -c / (di * dn);
      it.flow_next = J.flow(i + 1);
    }
  }
  it.w_self = (float)(k2 * w_self);
  it.w_prev = (float)(k2 * w_prev);
  it.w_next = (float)(k2 * w_next);
}

// Deterministic jobs' part of a scatter launch: the job's tiles in it (the
// blocks that share its scale) and a slot of its own, the reduce-only pass
// before the launch and the fold of the fixed-point fields after it.
struct DetLaunch {
  std::map<Job*, int> tiles;   // per deterministic job, its tiles in the launch
  std::map<Job*, int> slot;
};

template <class Item>
void det_assign(DetLaunch& dl, std::vector<Item>& items, const std::vector<Job*>& owner,
                std::map<Job*, int>& next_slot) {
  for (size_t k = 0; k < items.size(); ++k) {
    Job* J = owner[k];
    if (!J->det()) continue;
    const int* d = J->ldims[J->level];
    dl.tiles[J] += point_tiles(d[0], d[1], d[2]);
  }
  for (auto& kv : dl.tiles) {
    if (next_slot[kv.first] >= DET_SLOTS) fail(MUSTER_E_INTERNAL, "deterministic slots exhausted");
    dl.slot[kv.first] = next_slot[kv.first]++;
  }
}

template <class Item>
void add_det_stages(Builder& b, StageKind kind, const std::vector<Item>& items,
                    const std::vector<Job*>& owner, int staged,
                    const std::vector<DetFoldItem>& folds) {
  std::vector<Item> dmax;
  int tiles = 0;
  for (size_t k = 0; k < items.size(); ++k) {
    if (!owner[k]->det()) continue;
    Item it = items[k];
    it.tile0 = tiles;
    const int* d = owner[k]->ldims[owner[k]->level];
    tiles += point_tiles(d[0], d[1], d[2]);
    dmax.push_back(it);
  }
  b.add(kind, dmax, tiles, 0.0);
  if (!dmax.empty()) b.plan->stages.back().staged = staged;
  (void)folds;
}

void add_det_folds(Builder& b, std::vector<DetFoldItem>& folds) {
  int tiles = 0;
  for (DetFoldItem& f : folds) {
    f.tile0 = tiles;
    tiles += (f.n + ELEM_PER_BLOCK - 1) / ELEM_PER_BLOCK;
  }
  b.add(ST_DET_FOLD, folds, tiles, 0.0);
}

void add_backward(Builder& b, const std::vector<Job*>& jobs) {
  int maxK = 0, maxN = 0;
  std::vector<JobState*> det_states;
  std::map<Job*, int> next_slot;
  for (Job* J : jobs) {
    maxK = std::max(maxK, J->K());
    maxN = std::max(maxN, J->N);
    if (J->det()) det_states.push_back(J->js);
  }
  b.add(ST_DET_CLEAR, det_states, (int)det_states.size(), 0.0);
  add_sim_stages(b, jobs, ST_SIM_GRAD);
  add_rigid_stages(b, jobs);
  add_pair_resampling(b, jobs, true);
  for (int d = maxN - 1; d >= 2; --d) {
    std::vector<ComposeBwdItem> items;
    std::vector<Job*> owner;
    std::vector<int> gc_dir;
    int tiles = 0;
    double bytes = 0;
    for (Job* J : jobs) {
      const int N = J->N;
      if (d >= N) continue;
      const int* dd = J->ldims[J->level];
      for (int i = 0; i < N; ++i) {
        for (int j : {i + d, i - d}) {
          if (j < 0 || j >= N) continue;
          ComposeBwdItem it{};
          it.tile0 = tiles;
          it.D = dd[0]; it.H = dd[1]; it.W = dd[2];
          it.g = J->pair_grad(i, j);
          if (j > i) {
            it.prev = J->pair_field(i, j - 1);
            it.C = J->u_final(2 * (j - 1));
            it.gprev = J->pair_grad(i, j - 1);
            it.gc = J->pair_grad(j - 1, j);
          } else {
            it.prev = J->pair_field(i, j + 1);
            it.C = J->u_final(2 * j + 1);
            it.gprev = J->pair_grad(i, j + 1);
            it.gc = J->pair_grad(j + 1, j);
          }
          it.prev_atomic = (d == 2) ? 1 : 0;
          items.push_back(it);
          owner.push_back(J);
          gc_dir.push_back(j > i ? 2 * (j - 1) : 2 * j + 1);
          tiles += point_tiles(dd[0], dd[1], dd[2]);
          bytes += B_COMPOSE_BWD * J->Vc();
        }
      }
    }
    DetLaunch dl;
    det_assign(dl, items, owner, next_slot);
    std::vector<DetFoldItem> folds;
    for (size_t k = 0; k < items.size(); ++k) {
      Job* J = owner[k];
      if (!J->det()) continue;
      ComposeBwdItem& it = items[k];
      it.gc64 = J->det64_pair(gc_dir[k]);
      it.js = J->js;
      it.det_slot = dl.slot[J];
      it.det_blocks = dl.tiles[J];
      DetFoldItem f{};
      f.n = (int)(3 * J->Vc());
      f.f = it.gc;
      f.q = it.gc64;
      f.js = J->js;
      f.det_slot = it.det_slot;
      f.det_blocks = it.det_blocks;
      folds.push_back(f);
    }
    add_det_stages(b, ST_COMPOSE_BWD_DETMAX, items, owner, 0, folds);
    b.add(ST_COMPOSE_BWD, items, tiles, bytes);
    add_det_folds(b, folds);
  }
  for (int s = maxK - 1; s >= 0; --s) {
    // recompute u_s where needed
    if (s >= 1)
      for (int k = 0; k < s; ++k) add_exp_fwd_step(b, jobs, k, true, s);
    // one launch per staging mode in use (jobs with different K differ)
    std::vector<ExpBwdItem> items[4];
    std::vector<Job*> owner[4];
    int tiles[4] = {0, 0, 0, 0};
    double bytes[4] = {0, 0, 0, 0};
    for (Job* J : jobs) {
      const int K = J->K();
      if (s >= K) continue;
      const int* d = J->ldims[J->level];
      const float scale = std::ldexp(1.f, -K);
      // a staged G_0 is read by k_pull_combine or k_unstage
      const bool in_st = J->staged() && s < K - 1, out_st = J->staged();
      const int mode = in_st ? (out_st ? 2 : 3) : (out_st ? 1 : 0);
      for (int dir = 0; dir < 2 * (J->N - 1); ++dir) {
        const int i = dir / 2;
        const bool fwd = dir % 2 == 0;
        ExpBwdItem it{};
        it.tile0 = tiles[mode];
        it.D = d[0]; it.H = d[1]; it.W = d[2];
        if (s == 0) {
          it.src = J->flow(i);
          it.a = (fwd ? 1.f : -1.f) * scale;
        } else {
          it.src = J->u_step(dir, s);
          it.a = 1.f;
        }
        if (s == K - 1)
          it.gin = fwd ? J->pair_grad(i, i + 1) : J->pair_grad(i + 1, i);
        else
          it.gin = J->pp(dir, (s + 1) % 2);
        it.gout = J->pp(dir, s % 2);
        it.zero_in = (s < K - 1) ? 1 : 0;
        if (in_st) {
          it.stage_in = J->stage(dir, (s + 1) % 2);
          it.desc_in = J->desc(dir, (s + 1) % 2);
          it.flag_in = J->flag(dir, s + 1);
        }
        if (out_st) {
          it.stage_out = J->stage(dir, s % 2);
          it.desc_out = J->desc(dir, s % 2);
          it.flag_out = J->flag(dir, s);
        }
        // L_ss joins here unless k_pull_combine adds it (staged jobs)
        if (s == 0 && fwd && J->p.alpha_ss > 0.f && !J->staged()) {
          it.reg_w = std::ldexp(1.f, K) * J->p.alpha_ss / (float)(J->N - 1);
          it.reg_loss_w = J->p.alpha_ss / (float)(J->N - 1);
        }
        if (s == 0 && fwd) set_reg_ext(it, *J, i);
        it.js = J->js;
        if (J->det()) it.gout64 = J->det64_pp(dir, s % 2);
        items[mode].push_back(it);
        owner[mode].push_back(J);
        tiles[mode] += point_tiles(d[0], d[1], d[2]);
        bytes[mode] += B_EXP_BWD * J->Vc();
      }
    }
    for (int mode = 0; mode < 4; ++mode) {
      DetLaunch dl;
      det_assign(dl, items[mode], owner[mode], next_slot);
      std::vector<DetFoldItem> folds;
      bool any_det = false;
      for (size_t k = 0; k < items[mode].size(); ++k) {
        Job* J = owner[mode][k];
        if (!J->det()) continue;
        any_det = true;
        ExpBwdItem& it = items[mode][k];
        it.det_slot = dl.slot[J];
        it.det_blocks = dl.tiles[J];
        DetFoldItem f{};
        f.n = (int)(3 * J->Vc());
        f.f = it.gout;
        f.q = it.gout64;
        f.js = J->js;
        // staged out: only blocks that did not stage added into the flat field,
        // and each of them raised the flag
        f.flag = (mode == 1 || mode == 2) ? it.flag_out : nullptr;
        f.det_slot = it.det_slot;
        f.det_blocks = it.det_blocks;
        folds.push_back(f);
      }
      add_det_stages(b, ST_EXP_BWD_DETMAX, items[mode], owner[mode], mode, folds);
      b.add(ST_EXP_BWD, items[mode], tiles[mode], bytes[mode]);
      if (items[mode].empty()) continue;
      b.plan->stages.back().staged = mode;
      // deterministic jobs always run the general variant, so that their
      // arithmetic does not depend on the other jobs of the launch
      if (any_det) b.plan->stages.back().reg = 1;
      for (const ExpBwdItem& e : items[mode])
        if (e.reg_w != 0.f || e.ext) b.plan->stages.back().reg = 1;
      add_det_folds(b, folds);
    }
  }
  {
    // staged G_0 of both directions straight into the combined gradient t1,
    // with the diffusion regulariser (which the Exp adjoint's step 0 then
    // need not carry); Adam, or the smoothing of the gradient, reads t1
    std::vector<PullItem> pitems;
    std::vector<ExpBwdItem> uitems;
    int ptiles = 0, utiles = 0;
    double pbytes = 0, ubytes = 0;
    for (Job* J : jobs) {
      if (!J->staged()) continue;
      const int* d = J->ldims[J->level];
      const int pt = point_tiles(d[0], d[1], d[2]);
      for (int i = 0; i < J->N - 1; ++i) {
        if (J->staged()) {
          PullItem it{};
          it.tile0 = ptiles;
          it.D = d[0]; it.H = d[1]; it.W = d[2];
          for (int k = 0; k < 2; ++k) {
            const int dir = 2 * i + k;
            it.stage[k] = J->stage(dir, 0);
            it.desc[k] = J->desc(dir, 0);
            it.flag[k] = J->flag(dir, 0);
            it.gflat[k] = J->pp(dir, 0);
          }
          it.out = J->field(J->m_t1.as<float>(), i);
          it.scale = std::ldexp(1.f, -J->K());
          if (J->p.alpha_ss > 0.f) {
            it.reg_w = it.reg_loss_w = J->p.alpha_ss / (float)(J->N - 1);
            it.flow = J->flow(i);
            it.js = J->js;
          }
          pitems.push_back(it);
          ptiles += pt;
          // the two staged G_0, the gradient written, and the flow the
          // regulariser reads
          pbytes += (2 * B_UNSTAGE + (it.reg_w != 0.f ? 12 : 0)) * J->Vc();
        } else {
          for (int k = 0; k < 2; ++k) {
            const int dir = 2 * i + k;
            ExpBwdItem it{};
            it.tile0 = utiles;
            it.D = d[0]; it.H = d[1]; it.W = d[2];
            it.gout = J->pp(dir, 0);
            it.stage_in = J->stage(dir, 0);
            it.desc_in = J->desc(dir, 0);
            it.flag_in = J->flag(dir, 0);
            uitems.push_back(it);
            utiles += pt;
            ubytes += B_UNSTAGE * J->Vc();
          }
        }
      }
    }
    b.add(ST_PULL_COMBINE, pitems, ptiles, pbytes);
    b.add(ST_UNSTAGE, uitems, utiles, ubytes);
  }
  {
    // gradients of smoothing jobs: combine into t1 (staged jobs did above),
    // then smooth t1 -> t2 -> t1 -> t2
    std::vector<AdamItem> items;
    int tiles = 0;
    double bytes = 0;
    for (Job* J : jobs) {
      if (!J->smoothing() || J->staged()) continue;
      const size_t V = J->Vc();
      for (int i = 0; i < J->N - 1; ++i) {
        AdamItem it{};
        it.tile0 = tiles;
        it.n = (int)V;
        it.g0f = J->pp(2 * i, 0);
        it.g0b = J->pp(2 * i + 1, 0);
        it.gout = J->field(J->m_t1.as<float>(), i);
        it.scale = std::ldexp(1.f, -J->K());
        it.mode = 2;
        items.push_back(it);
        tiles += elem_tiles(V);
        bytes += 36.0 * V;
      }
    }
    b.add(ST_ADAM, items, tiles, bytes);
    auto t1 = [](Job* J, int i) { return J->field(J->m_t1.as<float>(), i); };
    auto t2 = [](Job* J, int i) { return J->field(J->m_t2.as<float>(), i); };
    add_smooth_pass(b, jobs, 0, [&](Job* J, int i) { return (const float*)t1(J, i); }, t2);
    add_smooth_pass(b, jobs, 1, [&](Job* J, int i) { return (const float*)t2(J, i); }, t1);
    add_smooth_pass(b, jobs, 2, [&](Job* J, int i) { return (const float*)t1(J, i); }, t2);
  }
  {
    std::vector<AdamItem> items;
    int tiles = 0;
    double bytes = 0;
    for (Job* J : jobs) {
      const size_t V = J->Vc();
      for (int i = 0; i < J->N - 1; ++i) {
        AdamItem it{};
        it.tile0 = tiles;
        it.n = (int)V;
        it.phi = J->field(J->phi, i);
        it.g0f = J->pp(2 * i, 0);
        it.g0b = J->pp(2 * i + 1, 0);
        it.gsrc = J->smoothing() ? J->field(J->m_t2.as<float>(), i)
                  : J->staged()  ? J->field(J->m_t1.as<float>(), i)
                                 : nullptr;
        it.m = J->field(J->mbuf, i);
        it.v = J->field(J->vbuf, i);
        it.scale = std::ldexp(1.f, -J->K());
        it.mode = J->grad_mode ? 1 : 0;
        it.gout = J->grad_mode ? J->grad_out + (size_t)i * 3 * V : nullptr;
        it.gscale = J->grad_scale;
        it.js = J->js;
        items.push_back(it);
        tiles += elem_tiles(V);
        bytes += B_ADAM * V;
      }
    }
    b.add(ST_ADAM, items, tiles, bytes);
  }
}

}  // namespace

std::unique_ptr<Plan> build_plan(const std::vector<Job*>& jobs, PlanScope scope) {
  auto plan = std::make_unique<Plan>();
  Builder b{plan.get()};
  if (jobs.empty()) return plan;
  const int window = jobs[0]->p.window, metric = jobs[0]->p.metric;
  for (Job* J : jobs)
    if (J->p.window != window || J->p.metric != metric)
      fail(MUSTER_E_INVALID, "jobs batched together must share window and metric");
  if (scope == PLAN_ITERATION || scope == PLAN_FORWARD || scope == PLAN_LOSS_FWD) add_forward(b, jobs);
  if (scope == PLAN_ITERATION || scope == PLAN_LOSS_FWD) add_sim_stages(b, jobs, ST_SIM_STATS);
  if (scope == PLAN_ITERATION || scope == PLAN_LOSS_BWD) add_backward(b, jobs);
  if (scope == PLAN_ITERATION) {
    std::vector<JobState*> st;
    for (Job* J : jobs) st.push_back(J->js);
    b.add(ST_FINISH, st, (int)st.size(), 0.0);
  }
  return plan;
}

Plan::~Plan() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
}

void Plan::upload(Ctx* ctx, hipStream_t s) {
  if (blob.empty()) return;
  dev.alloc(ctx, blob.size());
  MUSTER_HIP(hipMemcpyAsync(dev.p, blob.data(), blob.size(), hipMemcpyHostToDevice, s));
  MUSTER_HIP(hipStreamSynchronize(s));
}

static int kclass(StageKind k) {
  switch (k) {
    case ST_EXP_FWD: return MUSTER_K_EXP_FWD;
    case ST_COMPOSE_FWD: return MUSTER_K_COMPOSE_FWD;
    case ST_SIM_STATS: return MUSTER_K_SIM_STATS;
    case ST_SIM_GRAD: return MUSTER_K_SIM_GRAD;
    case ST_COMPOSE_BWD: return MUSTER_K_COMPOSE_BWD;
    case ST_EXP_BWD: return MUSTER_K_EXP_BWD;
    case ST_ADAM: return MUSTER_K_ADAM;
    case ST_FINISH: return MUSTER_K_FINISH;
    case ST_SMOOTH: return MUSTER_K_SMOOTH;
    case ST_UPSAMPLE: return MUSTER_K_UPSAMPLE;
    case ST_UPSAMPLE_ADJ: return MUSTER_K_UPSAMPLE_ADJ;
    case ST_RIGID_GRAD: return MUSTER_K_RIGID;
    case ST_RIGID_STEP: return MUSTER_K_RIGID;
    case ST_WARP: return MUSTER_K_WARP;
    case ST_UNSTAGE: return MUSTER_K_UNSTAGE;
    case ST_PULL_COMBINE: return MUSTER_K_UNSTAGE;
    case ST_COMPOSE_BWD_DETMAX: return MUSTER_K_COMPOSE_BWD;
    case ST_EXP_BWD_DETMAX: return MUSTER_K_EXP_BWD;
    case ST_DET_FOLD: return MUSTER_K_FINISH;
    case ST_DET_CLEAR: return MUSTER_K_FINISH;
  }
  return MUSTER_K_FINISH;
}

static hipError_t launch_stage(const Stage& st, const unsigned char* base, hipStream_t s) {
  const void* p = base + st.off;
  switch (st.kind) {
    case ST_EXP_FWD: return launch_exp_fwd((const ExpFwdItem*)p, st.n_items, st.n_tiles, s);
    case ST_COMPOSE_FWD: return launch_compose_fwd((const ComposeItem*)p, st.n_items, st.n_tiles, s);
    case ST_SIM_STATS:
      return launch_sim_stats((const SimItem*)p, st.n_items, st.n_tiles, st.window, st.metric,
                              st.shape, s);
    case ST_SIM_GRAD:
      return launch_sim_grad((const SimItem*)p, st.n_items, st.n_tiles, st.window, st.shape, s);
    case ST_COMPOSE_BWD:
      return launch_compose_bwd((const ComposeBwdItem*)p, st.n_items, st.n_tiles, s);
    case ST_EXP_BWD:
      return launch_exp_bwd((const ExpBwdItem*)p, st.n_items, st.n_tiles, st.staged, st.reg != 0, s);
    case ST_ADAM: return launch_adam((const AdamItem*)p, st.n_items, st.n_tiles, s);
    case ST_FINISH: return launch_finish((JobState* const*)p, st.n_items, s);
    case ST_SMOOTH: return launch_smooth((const SmoothItem*)p, st.n_items, st.n_tiles, st.lds, s);
    case ST_UPSAMPLE: return launch_upsample2((const UpItem*)p, st.n_items, st.n_tiles, s);
    case ST_UPSAMPLE_ADJ: return launch_upsample2_adj((const UpItem*)p, st.n_items, st.n_tiles, s);
    case ST_RIGID_GRAD:
      return launch_rigid_grad((const RigidGradItem*)p, st.n_items, st.n_tiles, s);
    case ST_RIGID_STEP: return launch_rigid_step((const RigidStepItem*)p, st.n_items, s);
    case ST_WARP: return launch_warp((const SimItem*)p, st.n_items, st.n_tiles, s);
    case ST_UNSTAGE: return launch_unstage((const ExpBwdItem*)p, st.n_items, st.n_tiles, s);
    case ST_PULL_COMBINE:
      return launch_pull_combine((const PullItem*)p, st.n_items, st.n_tiles, s);
    case ST_COMPOSE_BWD_DETMAX:
      return launch_compose_bwd_detmax((const ComposeBwdItem*)p, st.n_items, st.n_tiles, s);
    case ST_EXP_BWD_DETMAX:
      return launch_exp_bwd_detmax((const ExpBwdItem*)p, st.n_items, st.n_tiles, st.staged, s);
    case ST_DET_FOLD: return launch_det_fold((const DetFoldItem*)p, st.n_items, st.n_tiles, s);
    case ST_DET_CLEAR: return launch_det_clear((JobState* const*)p, st.n_items, s);
  }
  return hipErrorInvalidValue;
}

static void resolve_timing(Ctx* ctx) {
  std::lock_guard<std::mutex> lk(ctx->timing_mu);
  for (auto& t : ctx->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(t.b) == hipSuccess && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      ctx->stats.launches[t.k] += 1;
      ctx->stats.ms[t.k] += ms;
      ctx->stats.bytes[t.k] += t.bytes;
    }
    ctx->event_pool.push_back(t.a);
    ctx->event_pool.push_back(t.b);
  }
  ctx->pending.clear();
}

static hipEvent_t pooled_event(Ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  MUSTER_HIP(hipEventCreate(&e));
  return e;
}

void Plan::run(Ctx* ctx, hipStream_t s) {
  const unsigned char* base = dev.as<unsigned char>();
  for (const Stage& st : stages) {
    if (ctx->timing && ((ctx->timing_mask >> kclass(st.kind)) & 1u)) {
      std::lock_guard<std::mutex> lk(ctx->timing_mu);
      TimedLaunch t{};
      t.k = kclass(st.kind);
      t.bytes = st.bytes;
      t.a = pooled_event(ctx);
      t.b = pooled_event(ctx);
      set_launch_events(t.a, t.b);
      const hipError_t e = launch_stage(st, base, s);
      set_launch_events(nullptr, nullptr);
      MUSTER_HIP(e);
      ctx->pending.push_back(t);
    } else {
      MUSTER_HIP(launch_stage(st, base, s));
    }
  }
}

void Plan::capture(Ctx* ctx, hipStream_t s) {
  const unsigned char* base = dev.as<unsigned char>();
  MUSTER_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipSuccess;
  for (const Stage& st : stages) {
    err = launch_stage(st, base, s);
    if (err != hipSuccess) break;
  }
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(s, &g);
  MUSTER_HIP(err);
  MUSTER_HIP(e2);
  graph = g;
  MUSTER_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  (void)ctx;
}

void Plan::replay(hipStream_t s) { MUSTER_HIP(hipGraphLaunch(exec, s)); }

// ---------------------------------------------------------------------------
// batched registration engine (one or many jobs in lockstep)
// ---------------------------------------------------------------------------
static void run_level(Ctx* ctx, std::vector<Job*>& jobs, int level, hipStream_t s, bool use_graph) {
  const int T = jobs[0]->p.iters[level];
  Range range("muster level %d: %zu jobs, %d steps, %dx%dx%d", level, jobs.size(), T,
              jobs[0]->idims[level][0], jobs[0]->idims[level][1], jobs[0]->idims[level][2]);
  for (Job* J : jobs) job_begin_level(*J, level, s);
  if (T <= 0) return;
  auto plan = build_plan(jobs, PLAN_ITERATION);
  plan->upload(ctx, s);
  MUSTER_HIP(hipStreamSynchronize(s));
  const double t0 = now_seconds();
  if (use_graph && !ctx->timing) {
    plan->capture(ctx, s);
    for (int t = 0; t < T; ++t) plan->replay(s);
  } else {
    for (int t = 0; t < T; ++t) plan->run(ctx, s);
  }
  MUSTER_HIP(hipStreamSynchronize(s));
  const double dt = now_seconds() - t0;
  for (Job* J : jobs) J->step_seconds += dt;
  if (ctx->timing) resolve_timing(ctx);
  for (Job* J : jobs) read_state(*J, s);
}

static void fill_report(Job& J, double t0, muster_report* rep, hipStream_t s) {
  if (!rep) return;
  std::vector<double> h(std::max(J.hist_len, 1), 0.0);
  if (J.hist_len > 0) {
    MUSTER_HIP(hipMemcpyAsync(h.data(), J.hist, J.hist_len * sizeof(double), hipMemcpyDeviceToHost, s));
    MUSTER_HIP(hipStreamSynchronize(s));
  }
  rep->status = J.host_state->nonfinite ? MUSTER_E_NONFINITE : MUSTER_OK;
  rep->iterations = J.hist_len;
  rep->loss_first = J.hist_len > 0 ? h[0] : 0.0;
  rep->loss_last = J.hist_len > 0 ? h[J.hist_len - 1] : 0.0;
  rep->seconds = now_seconds() - t0;
  rep->queue_seconds = 0.0;
  rep->footprint_bytes = J.footprint;
  rep->step_seconds = J.step_seconds;
}

static void register_jobs(Ctx* ctx, hipStream_t caller, std::vector<std::unique_ptr<Job>>& owned,
                          muster_report* reports) {
  const double t0 = now_seconds();
  hipStream_t s = ctx->ws;
  hipEvent_t ev;
  MUSTER_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  MUSTER_HIP(hipEventRecord(ev, caller));
  MUSTER_HIP(hipStreamWaitEvent(s, ev, 0));
  (void)hipEventDestroy(ev);
  std::vector<Job*> jobs;
  for (auto& j : owned) jobs.push_back(j.get());
  const muster_params& p = jobs[0]->p;
  for (int l = 0; l < p.levels; ++l) run_level(ctx, jobs, l, s, p.use_graph != 0);
  for (Job* J : jobs) job_final_outputs(*J, s);
  bool bad = false;
  for (size_t k = 0; k < jobs.size(); ++k) {
    fill_report(*jobs[k], t0, reports ? &reports[k] : nullptr, s);
    if (jobs[k]->host_state->nonfinite) bad = true;
  }
  if (bad) fail(MUSTER_E_NONFINITE, "the loss of a job became non-finite");
}

// ---------------------------------------------------------------------------
// serving
// ---------------------------------------------------------------------------
// The server's executor: jobs, launch plans (one per group of residents that
// share window, metric and K, rebuilt when its members or levels change) and
// kernels on the serving thread's own stream.
namespace {
struct HipJob : JobHandle {
  std::unique_ptr<Job> job;
};

Job& job_of(JobHandle& h) { return *static_cast<HipJob&>(h).job; }

struct HipExecutor : Executor {
  Ctx* ctx;
  hipStream_t s = nullptr;
  std::map<GroupKey, std::unique_ptr<Plan>> plans;
  std::map<GroupKey, std::vector<std::pair<uint64_t, int>>> sigs;
  explicit HipExecutor(Ctx* c) : ctx(c) {}
  uint64_t footprint(const muster_job& j) override {
    return job_footprint(j.N, j.dims, j.params);
  }
  uint64_t budget() override { return ctx->arena.budget(); }
  bool fits(uint64_t bytes) override { return ctx->arena.fits(bytes); }
  std::unique_ptr<JobHandle> admit(const muster_job& j) override {
    Range range("muster admit job: N %d", j.N);
    auto h = std::make_unique<HipJob>();
    h->job = make_job(ctx, j);
    job_begin_level(*h->job, 0, s);
    return h;
  }
  void step(const GroupKey& key, const std::vector<JobHandle*>& group,
            const std::vector<std::pair<uint64_t, int>>& sig) override {
    std::unique_ptr<Plan>& plan = plans[key];
    if (!plan || sigs[key] != sig) {
      std::vector<Job*> jobs;
      for (JobHandle* h : group) jobs.push_back(&job_of(*h));
      plan = build_plan(jobs, PLAN_ITERATION);
      plan->upload(ctx, s);
      sigs[key] = sig;
    }
    plan->run(ctx, s);
  }
  void forget_groups_except(const std::vector<GroupKey>& live) override {
    for (auto it = plans.begin(); it != plans.end();) {
      if (std::find(live.begin(), live.end(), it->first) == live.end()) {
        sigs.erase(it->first);
        it = plans.erase(it);
      } else {
        ++it;
      }
    }
  }
  void sync(const std::vector<JobHandle*>& resident) override {
    Range range("muster server tick: %zu resident", resident.size());
    for (JobHandle* h : resident) {
      Job& J = job_of(*h);
      MUSTER_HIP(hipMemcpyAsync(J.host_state, J.js, sizeof(JobState), hipMemcpyDeviceToHost, s));
    }
    MUSTER_HIP(hipStreamSynchronize(s));
  }
  int level(JobHandle& h) override { return job_of(h).level; }
  bool nonfinite(JobHandle& h) override { return job_of(h).host_state->nonfinite != 0; }
  void begin_level(JobHandle& h, int level) override { job_begin_level(job_of(h), level, s); }
  void finish(JobHandle& h, double t_submit, muster_report* rep) override {
    job_final_outputs(job_of(h), s);
    fill_report(job_of(h), t_submit, rep, s);
  }
  uint64_t held_bytes(JobHandle& h) override { return job_of(h).footprint; }
  void on_device_error() override { ctx->poisoned = true; }
};
}  // namespace

Server::Server(Ctx* c, int max_queue) : ctx(c) {
  ex = std::make_unique<HipExecutor>(c);
  sched = std::make_unique<Scheduler>(*ex, max_queue, now_seconds);
}

Server::~Server() {
  sched->stop();
  if (th.joinable()) th.join();
}

void Server::loop() {
  auto* hx = static_cast<HipExecutor*>(ex.get());
  if (hipSetDevice(ctx->device) != hipSuccess ||
      hipStreamCreateWithFlags(&hx->s, hipStreamNonBlocking) != hipSuccess) {
    sched->stop();
    sched->shutdown();
    return;
  }
  while (sched->wait_for_work()) sched->tick();
  sched->shutdown();
  hx->plans.clear();
  hx->sigs.clear();
  (void)hipStreamSynchronize(hx->s);
  (void)hipStreamDestroy(hx->s);
  hx->s = nullptr;
}


// ---------------------------------------------------------------------------
// Autotuner of the window-statistics tiling.  Each candidate (tile shape,
// z chunk) runs the statistics and gradient kernels on a scratch problem of
// the same shape (two patterned images and a patterned pair field), one
// untimed and three timed repetitions; the fastest median wins.  Results are
// kept per context and, with MUSTER_TUNE_CACHE set, appended to that file and
// read back by later contexts.
// ---------------------------------------------------------------------------
namespace {

std::vector<int> tune_key(const int d[3], int window, int metric) {
  return {d[0], d[1], d[2], window, metric};
}

void save_tune_entry(Ctx* ctx, const std::vector<int>& k, const SimTile& t) {
  if (ctx->tune_path.empty()) return;
  FILE* f = std::fopen(ctx->tune_path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %d %d %d %d\n", k[0], k[1], k[2], k[3], k[4], t.shape, t.zc);
  std::fclose(f);
}

SimTile default_sim_tile(const int dims[3]) {
  SimTile t;
  t.shape = 0;
  t.zc = std::min(32, dims[0]);
  return t;
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    MUSTER_HIP(hipEventCreate(&a));
    MUSTER_HIP(hipEventCreate(&b));
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

SimTile tune_sim_tile(Ctx* ctx, const int dims[3], int window, int metric, hipStream_t s) {
  // A launch of the real path carries every pair of a job (6 to 90), so the
  // scratch launch carries several pairs with distinct fields, as many as
  // fit 1.5 GB, at most 8.
  const size_t V = (size_t)dims[0] * dims[1] * dims[2];
  const size_t per_pair = 9 * V * sizeof(float);
  const int P = (int)std::max<size_t>(1, std::min<size_t>(8, ((size_t)1536 << 20) / per_pair));
  DevMem img, fld, acc, item;
  img.alloc(ctx, 2 * V * sizeof(float));
  fld.alloc(ctx, (size_t)P * per_pair);
  acc.alloc(ctx, sizeof(double));
  item.alloc(ctx, (size_t)P * sizeof(SimItem));
  MUSTER_HIP(launch_pattern(img.as<float>(), (int64_t)(2 * V), dims, 0.5f, 0.4f, 0.3f, s));
  MUSTER_HIP(launch_pattern(fld.as<float>(), (int64_t)(9 * V * P), dims, 0.f, 1.5f, 1.1f, s));
  const int r = (window - 1) / 2;
  std::vector<SimItem> its(P);
  for (int k = 0; k < P; ++k) {
    SimItem& it = its[k];
    float* base = fld.as<float>() + (size_t)k * 9 * V;
    it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
    it.F = img.as<float>();
    it.I = img.as<float>() + V;
    it.U = base;
    it.coef = base + 3 * V;
    it.gU = base + 6 * V;
    it.M = it.gU;
    it.inv_nr = 1.0 / ((double)(dims[0] - 2 * r) * (dims[1] - 2 * r) * (dims[2] - 2 * r));
    it.js = nullptr;
    it.sim_out = acc.as<double>();
  }
  // the warp does not depend on the tiling: once, before the timed stages
  {
    const int pt = point_tiles(dims[0], dims[1], dims[2]);
    for (int k = 0; k < P; ++k) its[k].tile0 = k * pt;
    MUSTER_HIP(hipMemcpyAsync(item.p, its.data(), (size_t)P * sizeof(SimItem),
                              hipMemcpyHostToDevice, s));
    MUSTER_HIP(launch_warp(item.as<SimItem>(), P, P * pt, s));
  }
  std::vector<int> zcs;
  for (int z : {16, 32, 64}) {
    const int zc = std::min(z, dims[0]);
    if (std::find(zcs.begin(), zcs.end(), zc) == zcs.end()) zcs.push_back(zc);
  }
  EventPair ev;
  SimTile best = default_sim_tile(dims);
  float best_ms = 1e30f;
  for (int shape = 0; shape < SIM_SHAPES; ++shape)
    for (int zc : zcs) {
      const int per = stat_tiles(dims[0], dims[1], dims[2], zc, shape);
      for (int k = 0; k < P; ++k) {
        its[k].zc = zc;
        its[k].tile0 = k * per;
      }
      MUSTER_HIP(hipMemcpyAsync(item.p, its.data(), (size_t)P * sizeof(SimItem),
                                hipMemcpyHostToDevice, s));
      const SimItem* d_it = item.as<SimItem>();
      auto once = [&] {
        MUSTER_HIP(launch_sim_stats(d_it, P, P * per, window, metric, shape, s));
        MUSTER_HIP(launch_sim_grad(d_it, P, P * per, window, shape, s));
      };
      once();
      float t[3];
      for (float& x : t) {
        MUSTER_HIP(hipEventRecord(ev.a, s));
        once();
        MUSTER_HIP(hipEventRecord(ev.b, s));
        MUSTER_HIP(hipEventSynchronize(ev.b));
        MUSTER_HIP(hipEventElapsedTime(&x, ev.a, ev.b));
      }
      std::sort(t, t + 3);
      if (std::getenv("MUSTER_TUNE_VERBOSE"))
        std::fprintf(stderr, "muster tune %dx%dx%d w%d m%d (%d pairs): shape %d zchunk %d  %.4f ms\n",
                     dims[0], dims[1], dims[2], window, metric, P, shape, zc, (double)t[1]);
      if (t[1] < best_ms) {
        best_ms = t[1];
        best.shape = shape;
        best.zc = zc;
      }
    }
  MUSTER_HIP(hipStreamSynchronize(s));
  return best;
}

}  // namespace

void load_tune_cache(Ctx* ctx) {
  const char* path = std::getenv("MUSTER_TUNE_CACHE");
  if (!path || !*path) return;
  ctx->tune_path = path;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  int D, H, W, w, m, sh, zc;
  while (std::fscanf(f, "%d %d %d %d %d %d %d", &D, &H, &W, &w, &m, &sh, &zc) == 7)
    if (sh >= 0 && sh < SIM_SHAPES && zc >= 1 && zc <= D) ctx->tuned[{D, H, W, w, m}] = SimTile{sh, zc};
  std::fclose(f);
}

SimTile choose_sim_tile(Ctx* ctx, const int dims[3], int window, int metric, hipStream_t s) {
  if (ctx->tile_mode == MUSTER_TILES_DEFAULT) return default_sim_tile(dims);
  if (ctx->tile_mode == MUSTER_TILES_FIXED) {
    SimTile t = ctx->fixed_tile;
    t.zc = std::min(t.zc, dims[0]);
    return t;
  }
  const auto key = tune_key(dims, window, metric);
  {
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    auto f = ctx->tuned.find(key);
    if (f != ctx->tuned.end()) return f->second;
  }
  SimTile t;
  try {
    t = tune_sim_tile(ctx, dims, window, metric, s);
  } catch (const Error& e) {
    if (e.st != MUSTER_E_NOMEM) throw;
    return default_sim_tile(dims);  // no room for the scratch problem now: do not cache
  }
  std::lock_guard<std::mutex> lk(ctx->tune_mu);
  if (ctx->tuned.emplace(key, t).second) save_tune_entry(ctx, key, t);
  return t;
}

}  // namespace muster

// ===========================================================================
// C ABI
// ===========================================================================
using namespace muster;

struct muster_ctx {
  Ctx* c;
};

struct muster_saved {
  muster_ctx* ctx;
  std::unique_ptr<Job> job;
  bool used = false;
};

static Ctx* C(muster_ctx* h) { return h ? h->c : nullptr; }

#define NEED(cond, ...) \
  do {                  \
    if (!(cond)) fail(MUSTER_E_INVALID, __VA_ARGS__); \
  } while (0)

namespace {

struct StepCall {
  Ctx* ctx;
  hipStream_t s;
  std::vector<unsigned char> blob;
  template <class Item>
  size_t add(const Item& it) {
    size_t off = (blob.size() + 63) & ~(size_t)63;
    blob.resize(off + sizeof(Item));
    std::memcpy(blob.data() + off, &it, sizeof(Item));
    return off;
  }
  const unsigned char* dev() const { return (const unsigned char*)ctx->step_items; }
  void upload() {
    NEED(blob.size() <= ctx->step_items_bytes, "too many steps for one call");
    if (!blob.empty())
      MUSTER_HIP(hipMemcpyAsync(ctx->step_items, blob.data(), blob.size(), hipMemcpyHostToDevice, s));
  }
};

void check_dims(const int dims[3], int min_edge) {
  NEED(dims, "dims is NULL");
  uint64_t V = 1;
  for (int d = 0; d < 3; ++d) {
    NEED(dims[d] >= min_edge, "dims[%d] = %d must be at least %d", d, dims[d], min_edge);
    V *= (uint64_t)dims[d];
  }
  NEED(V * 3 < (uint64_t)INT32_MAX, "volume too large");
}

}  // namespace

extern "C" {

const char* muster_last_error(void) { return g_err.c_str(); }
const char* muster_version(void) { return "muster-mi355x 0.1.0 (gfx950)"; }

muster_status muster_ctx_create(int device, uint64_t hbm_budget, muster_ctx** out) {
  return guard(nullptr, [&] {
    NEED(out, "out is NULL");
    int n = 0;
    MUSTER_HIP(hipGetDeviceCount(&n));
    NEED(device >= 0 && device < n, "device %d out of range (%d devices)", device, n);
    MUSTER_HIP(hipSetDevice(device));
    if (hbm_budget == 0) {
      // no bound given: 80 % of what is free on the device now, so that
      // admission by footprint never runs the device out of memory
      size_t free_b = 0, total_b = 0;
      MUSTER_HIP(hipMemGetInfo(&free_b, &total_b));
      hbm_budget = (uint64_t)(0.8 * (double)free_b);
    }
    auto c = std::make_unique<Ctx>(hbm_budget, device);
    c->device = device;
    // the allocation-free entry point's scratch on this device (current now)
    MUSTER_HIP(noalloc_scratch_address(device, &c->noalloc_scratch));
    load_tune_cache(c.get());
    MUSTER_HIP(hipStreamCreateWithFlags(&c->ws, hipStreamNonBlocking));
    c->step_items_bytes = 1 << 20;
    c->step_items = c->arena.try_alloc(c->step_items_bytes);
    c->step_acc = (double*)c->arena.try_alloc(64 * sizeof(double));
    NEED(c->step_items && c->step_acc, "could not allocate context buffers");
    *out = new muster_ctx{c.release()};
  });
}

muster_status muster_ctx_destroy(muster_ctx* h) {
  if (!h) return MUSTER_OK;
  Ctx* c = h->c;
  if (c->server) c->server.reset();  // stops the serving thread and fails what is left
  (void)hipSetDevice(c->device);
  if (c->ws) {
    (void)hipStreamSynchronize(c->ws);
    (void)hipStreamDestroy(c->ws);
  }
  if (c->step_items) c->arena.release(c->step_items);
  if (c->step_acc) c->arena.release(c->step_acc);
  for (auto& t : c->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  delete c;
  delete h;
  return MUSTER_OK;
}

muster_status muster_params_default(muster_params* p) {
  return guard(nullptr, [&] {
    NEED(p, "params is NULL");
    std::memset(p, 0, sizeof *p);
    p->levels = 1;
    p->iters[0] = 100;
    p->K = 7;
    p->window = 5;
    p->metric = MUSTER_METRIC_LNCC;
    p->alpha_ss = 1.0f;
    p->lr = 0.1f;
    p->warmup = 0.2f;
    p->beta1 = 0.9f;
    p->beta2 = 0.999f;
    p->eps = 1e-8f;
    p->exp_mode = MUSTER_EXP_STORE;
    p->use_graph = 1;
    p->smooth_sigma = 0.0f;
    p->flow_factor = 1;
  });
}

muster_status muster_footprint(int N, const int dims[3], const muster_params* p, uint64_t* bytes) {
  return guard(nullptr, [&] {
    NEED(p && bytes, "NULL argument");
    validate_problem(N, dims, *p, nullptr);
    *bytes = job_footprint(N, dims, *p);
  });
}

muster_status muster_register(muster_ctx* h, void* stream, int N, const int dims[3],
                              const float* images_dev, const double* times_host,
                              const muster_params* params, float* svf_out_dev,
                              float* pairs_out_dev, muster_report* report) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx, "ctx is NULL");
    NEED(params, "params is NULL");
    NEED(images_dev && svf_out_dev, "images and svf_out must not be NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    muster_job jd{};
    jd.N = N;
    if (dims) std::memcpy(jd.dims, dims, sizeof jd.dims);
    jd.images_dev = images_dev;
    jd.times_host = times_host;
    jd.svf_out_dev = svf_out_dev;
    jd.pairs_out_dev = pairs_out_dev;
    jd.params = *params;
    NEED(dims, "dims is NULL");
    std::vector<std::unique_ptr<Job>> jobs;
    jobs.push_back(make_job(ctx, jd));
    register_jobs(ctx, (hipStream_t)stream, jobs, report);
  });
}

muster_status muster_register_batch(muster_ctx* h, void* stream, int n_jobs, const muster_job* jobs,
                                    muster_report* reports) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && jobs && n_jobs > 0, "bad arguments");
    std::lock_guard<std::mutex> lk(ctx->mu);
    const muster_params& p0 = jobs[0].params;
    for (int k = 0; k < n_jobs; ++k) {
      const muster_params& p = jobs[k].params;
      NEED(jobs[k].svf_out_dev, "job %d: svf_out is NULL", k);
      bool same = p.levels == p0.levels && p.K == p0.K && p.window == p0.window &&
                  p.metric == p0.metric;
      for (int l = 0; same && l < p.levels; ++l) same = p.iters[l] == p0.iters[l];
      NEED(same, "job %d: batched jobs must share levels, iters, K, window and metric", k);
    }
    std::vector<std::unique_ptr<Job>> owned;
    for (int k = 0; k < n_jobs; ++k) owned.push_back(make_job(ctx, jobs[k]));
    register_jobs(ctx, (hipStream_t)stream, owned, reports);
  });
}

muster_status muster_server_start(muster_ctx* h, int max_queue) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx, "ctx is NULL");
    NEED(max_queue > 0, "max_queue must be positive");
    NEED(!ctx->server, "server already running");
    ctx->server = std::make_unique<Server>(ctx, max_queue);
    Server* sv = ctx->server.get();
    sv->th = std::thread([sv] { sv->loop(); });
  });
}

muster_status muster_submit(muster_ctx* h, const muster_job* job, uint64_t* ticket) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && job && ticket, "NULL argument");
    NEED(ctx->server, "server not started");
    validate_problem(job->N, job->dims, job->params, job->times_host);
    NEED(job->images_dev && job->svf_out_dev, "images and svf_out must not be NULL");
    *ticket = ctx->server->sched->submit(*job);
  });
}

muster_status muster_poll(muster_ctx* h, uint64_t ticket, int* state) {
  Ctx* ctx = C(h);
  return guard(nullptr, [&] {
    NEED(ctx && ctx->server && state, "bad arguments");
    *state = ctx->server->sched->poll(ticket);
  });
}

muster_status muster_wait(muster_ctx* h, uint64_t ticket, muster_report* report) {
  Ctx* ctx = C(h);
  muster_status st = MUSTER_OK;
  std::string err;
  const muster_status g = guard(nullptr, [&] {
    NEED(ctx && ctx->server, "server not started");
    st = ctx->server->sched->wait(ticket, report, &err);
  });
  if (g != MUSTER_OK) return g;
  // keep the job's error text for the caller
  if (st != MUSTER_OK) set_error("%s", err.c_str());
  return st;
}

muster_status muster_cancel(muster_ctx* h, uint64_t ticket) {
  Ctx* ctx = C(h);
  return guard(nullptr, [&] {
    NEED(ctx && ctx->server, "server not started");
    ctx->server->sched->cancel(ticket);
  });
}

muster_status muster_server_stats(muster_ctx* h, int* resident, int* queued, uint64_t* bytes) {
  Ctx* ctx = C(h);
  return guard(nullptr, [&] {
    NEED(ctx && ctx->server, "server not started");
    ctx->server->sched->stats(resident, queued);
    if (bytes) *bytes = ctx->arena.used();
  });
}

// ---- autograd ---------------------------------------------------------------

muster_status muster_loss_forward(muster_ctx* h, void* stream, int N, const int dims[3],
                                  const float* images_dev, const double* times_host,
                                  const float* svf_dev, const muster_params* params,
                                  double* loss_host, muster_saved** saved) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && params && images_dev && svf_dev && loss_host && saved, "NULL argument");
    NEED(!params->rigid, "the rigid adjustment is available through the registration entry points only");
    NEED(dims, "dims is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t s = (hipStream_t)stream;
    muster_job jd{};
    jd.N = N;
    std::memcpy(jd.dims, dims, sizeof jd.dims);
    jd.images_dev = images_dev;
    jd.times_host = times_host;
    jd.params = *params;
    jd.params.levels = 1;
    jd.params.iters[0] = 0;
    auto job = make_job(ctx, jd);
    Job& J = *job;
    J.grad_mode = true;
    J.phi = const_cast<float*>(svf_dev);
    job_begin_level(J, 0, s);
    std::vector<Job*> one{&J};
    auto plan = build_plan(one, PLAN_LOSS_FWD);
    plan->upload(ctx, s);
    plan->run(ctx, s);
    const GridDims fd{J.ldims[0][0], J.ldims[0][1], J.ldims[0][2]};  // the flow grid
    for (int i = 0; i < N - 1; ++i)
      MUSTER_HIP(launch_reg(fd, J.flow(i), &J.js->loss_reg, nullptr, s));
    for (int i = 0; i < N - 1; ++i) {
      ExpBwdItem e{};
      set_reg_ext(e, J, i);
      if (e.ext)
        MUSTER_HIP(launch_reg_ext(fd, J.flow(i), e.flow_prev, e.l2_loss_w, e.ts_loss_w, e.inv_dprev,
                                  e.inv_dself, &J.js->loss_ext, s));
    }
    read_state(J, s);
    if (ctx->timing) resolve_timing(ctx);
    *loss_host = J.host_state->loss_sim +
                 (double)params->alpha_ss / (N - 1) * J.host_state->loss_reg + J.host_state->loss_ext;
    auto* sv = new muster_saved;
    sv->ctx = h;
    sv->job = std::move(job);
    *saved = sv;
  });
}

muster_status muster_loss_backward(muster_ctx* h, void* stream, muster_saved* saved,
                                   double grad_out, float* grad_svf_dev) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && saved && grad_svf_dev, "NULL argument");
    NEED(!saved->used, "saved state was already used by a backward pass");
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t s = (hipStream_t)stream;
    Job& J = *saved->job;
    J.grad_out = grad_svf_dev;
    J.grad_scale = (float)grad_out;
    std::vector<Job*> one{&J};
    auto plan = build_plan(one, PLAN_LOSS_BWD);
    plan->upload(ctx, s);
    plan->run(ctx, s);
    MUSTER_HIP(hipStreamSynchronize(s));
    if (ctx->timing) resolve_timing(ctx);
    saved->used = true;
  });
}

muster_status muster_saved_free(muster_saved* saved) {
  if (!saved) return MUSTER_OK;
  if (saved->ctx) (void)hipSetDevice(saved->ctx->c->device);
  delete saved;
  return MUSTER_OK;
}

// ---- single steps -------------------------------------------------------------


muster_status muster_exp(muster_ctx* h, void* stream, const int dims[3], int K, int sign,
                         const float* svf, float* disp, float* steps) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && svf && disp, "NULL argument");
    check_dims(dims, 2);
    NEED(K >= 1 && K <= 20, "K must be in 1..20");
    NEED(sign == 1 || sign == -1, "sign must be +1 or -1");
    std::lock_guard<std::mutex> lk(ctx->mu);
    StepCall sc{ctx, (hipStream_t)stream, {}};
    const size_t V = (size_t)dims[0] * dims[1] * dims[2];
    DevMem tmp;
    if (!steps) tmp.alloc(ctx, 2 * 3 * V * sizeof(float));
    auto buf = [&](int k) -> float* {  // u_k, k in 1..K-1
      if (steps) return steps + (size_t)(k - 1) * 3 * V;
      return tmp.as<float>() + (size_t)((k - 1) % 2) * 3 * V;
    };
    const int tiles = point_tiles(dims[0], dims[1], dims[2]);
    std::vector<size_t> offs;
    for (int s = 0; s < K; ++s) {
      ExpFwdItem it{};
      it.tile0 = 0;
      it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
      it.src = s == 0 ? svf : buf(s);
      it.a = s == 0 ? (float)sign * std::ldexp(1.f, -K) : 1.f;
      it.dst = s == K - 1 ? disp : buf(s + 1);
      offs.push_back(sc.add(it));
    }
    sc.upload();
    for (int s = 0; s < K; ++s)
      MUSTER_HIP(launch_exp_fwd((const ExpFwdItem*)(sc.dev() + offs[s]), 1, tiles, sc.s));
    if (steps)
      MUSTER_HIP(hipMemcpyAsync(steps + (size_t)(K - 1) * 3 * V, disp, 3 * V * sizeof(float),
                                hipMemcpyDeviceToDevice, sc.s));
    MUSTER_HIP(hipStreamSynchronize(sc.s));
  });
}

muster_status muster_exp_bwd(muster_ctx* h, void* stream, const int dims[3], int K, int sign,
                             const float* svf, const float* grad_disp, float* grad_svf, int mode) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && svf && grad_disp && grad_svf, "NULL argument");
    check_dims(dims, 2);
    NEED(K >= 1 && K <= 20, "K must be in 1..20");
    NEED(sign == 1 || sign == -1, "sign must be +1 or -1");
    const bool flat_only = (mode & MUSTER_EXP_FLAT) != 0;
    mode &= ~MUSTER_EXP_FLAT;
    NEED(mode == MUSTER_EXP_STORE || mode == MUSTER_EXP_RECOMPUTE, "bad mode");
    std::lock_guard<std::mutex> lk(ctx->mu);
    StepCall sc{ctx, (hipStream_t)stream, {}};
    const size_t V = (size_t)dims[0] * dims[1] * dims[2];
    const size_t F = 3 * V;
    const int nstore = mode == MUSTER_EXP_STORE ? std::max(K - 1, 0) : 2;
    const int tiles = point_tiles(dims[0], dims[1], dims[2]);
    // the squaring steps exchange their scatter boxes through staging slots,
    // as in the registration, unless the caller asks for the flat path
    const bool staged = !flat_only && K >= 2;
    DevMem us, pp, zero, stage, desc, flags;
    us.alloc(ctx, std::max<size_t>(nstore, 1) * F * sizeof(float));
    pp.alloc(ctx, 2 * F * sizeof(float));
    zero.alloc(ctx, F * sizeof(float));
    MUSTER_HIP(launch_fill(pp.as<float>(), (int64_t)(2 * F), 0.f, sc.s));
    MUSTER_HIP(launch_fill(zero.as<float>(), (int64_t)F, 0.f, sc.s));
    if (staged) {
      stage.alloc(ctx, (size_t)2 * tiles * 3 * STAGE_CAP * sizeof(float));
      desc.alloc(ctx, (size_t)2 * tiles * 8 * sizeof(int));
      flags.alloc(ctx, (size_t)K * sizeof(int));
      // zero bits: the overflow flags start clear
      MUSTER_HIP(launch_fill(flags.as<float>(), (int64_t)K, 0.f, sc.s));
    }
    auto st_slot = [&](int k) { return stage.as<float>() + (size_t)k * tiles * 3 * STAGE_CAP; };
    auto de_slot = [&](int k) { return desc.as<int>() + (size_t)k * tiles * 8; };
    const float a0 = (float)sign * std::ldexp(1.f, -K);
    auto ustore = [&](int k) { return us.as<float>() + (size_t)(k - 1) * F; };        // store: u_k
    auto uscr = [&](int k) { return us.as<float>() + (size_t)((k - 1) % 2) * F; };    // recompute
    struct L { int kind; size_t off; int smode; };
    std::vector<L> seq;
    auto fwd_step = [&](int k, float* src, float* dst) {
      ExpFwdItem it{};
      it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
      it.src = k == 0 ? svf : src;
      it.a = k == 0 ? a0 : 1.f;
      it.dst = dst;
      seq.push_back({0, sc.add(it), 0});
    };
    if (mode == MUSTER_EXP_STORE)
      for (int k = 0; k < K - 1; ++k) fwd_step(k, k == 0 ? nullptr : ustore(k), ustore(k + 1));
    for (int s = K - 1; s >= 0; --s) {
      const float* us_src;
      if (s == 0) {
        us_src = svf;
      } else if (mode == MUSTER_EXP_STORE) {
        us_src = ustore(s);
      } else {
        for (int k = 0; k < s; ++k) fwd_step(k, k == 0 ? nullptr : uscr(k), uscr(k + 1));
        us_src = uscr(s);
      }
      ExpBwdItem it{};
      it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
      it.src = us_src;
      it.a = s == 0 ? a0 : 1.f;
      it.gin = s == K - 1 ? const_cast<float*>(grad_disp) : pp.as<float>() + (size_t)((s + 1) % 2) * F;
      it.gout = pp.as<float>() + (size_t)(s % 2) * F;
      it.zero_in = s < K - 1 ? 1 : 0;
      const bool in_st = staged && s < K - 1;
      if (in_st) {
        it.stage_in = st_slot((s + 1) % 2);
        it.desc_in = de_slot((s + 1) % 2);
        it.flag_in = flags.as<int>() + s + 1;
      }
      if (staged) {
        it.stage_out = st_slot(s % 2);
        it.desc_out = de_slot(s % 2);
        it.flag_out = flags.as<int>() + s;
      }
      seq.push_back({1, sc.add(it), in_st ? 2 : (staged ? 1 : 0)});
    }
    if (staged) {
      // the staged G_0 to the flat field, as k_unstage does in the registration
      ExpBwdItem it{};
      it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
      it.gout = pp.as<float>();
      it.stage_in = st_slot(0);
      it.desc_in = de_slot(0);
      it.flag_in = flags.as<int>();
      seq.push_back({3, sc.add(it), 0});
    }
    AdamItem ai{};
    ai.n = (int)V;
    ai.g0f = pp.as<float>();
    ai.g0b = zero.as<float>();
    ai.gout = grad_svf;
    ai.scale = a0;
    ai.gscale = 1.f;
    ai.mode = 1;
    seq.push_back({2, sc.add(ai), 0});
    sc.upload();
    for (auto& l : seq) {
      const unsigned char* p = sc.dev() + l.off;
      if (l.kind == 0) MUSTER_HIP(launch_exp_fwd((const ExpFwdItem*)p, 1, tiles, sc.s));
      if (l.kind == 1) MUSTER_HIP(launch_exp_bwd((const ExpBwdItem*)p, 1, tiles, l.smode, false, sc.s));
      if (l.kind == 3) MUSTER_HIP(launch_unstage((const ExpBwdItem*)p, 1, tiles, sc.s));
      if (l.kind == 2) MUSTER_HIP(launch_adam((const AdamItem*)p, 1, elem_tiles(V), sc.s));
    }
    MUSTER_HIP(hipStreamSynchronize(sc.s));
  });
}

muster_status muster_compose(muster_ctx* h, void* stream, const int dims[3], const float* U_prev,
                             const float* Cf, float* out) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && U_prev && Cf && out, "NULL argument");
    check_dims(dims, 2);
    std::lock_guard<std::mutex> lk(ctx->mu);
    StepCall sc{ctx, (hipStream_t)stream, {}};
    ComposeItem it{};
    it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
    it.prev = U_prev;
    it.C = Cf;
    it.out = out;
    const size_t off = sc.add(it);
    sc.upload();
    MUSTER_HIP(launch_compose_fwd((const ComposeItem*)(sc.dev() + off), 1,
                                  point_tiles(dims[0], dims[1], dims[2]), sc.s));
    MUSTER_HIP(hipStreamSynchronize(sc.s));
  });
}

muster_status muster_compose_bwd(muster_ctx* h, void* stream, const int dims[3], const float* U_prev,
                                 const float* Cf, const float* G, float* G_prev, float* G_C) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && U_prev && Cf && G && G_prev && G_C, "NULL argument");
    check_dims(dims, 2);
    std::lock_guard<std::mutex> lk(ctx->mu);
    StepCall sc{ctx, (hipStream_t)stream, {}};
    ComposeBwdItem it{};
    it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
    it.g = G;
    it.prev = U_prev;
    it.C = Cf;
    it.gprev = G_prev;
    it.gc = G_C;
    it.prev_atomic = 1;
    const size_t off = sc.add(it);
    sc.upload();
    MUSTER_HIP(launch_compose_bwd((const ComposeBwdItem*)(sc.dev() + off), 1,
                                  point_tiles(dims[0], dims[1], dims[2]), sc.s));
    MUSTER_HIP(hipStreamSynchronize(sc.s));
  });
}

muster_status muster_sim(muster_ctx* h, void* stream, const int dims[3], int window, int metric,
                         const float* F, const float* I, const float* U, double* sim_host,
                         float* grad_U) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && F && I && U && sim_host, "NULL argument");
    NEED(window == 3 || window == 5 || window == 7, "window must be 3, 5 or 7");
    NEED(metric == MUSTER_METRIC_LNCC || metric == MUSTER_METRIC_SILNCC, "unknown metric");
    check_dims(dims, window);
    std::lock_guard<std::mutex> lk(ctx->mu);
    StepCall sc{ctx, (hipStream_t)stream, {}};
    const size_t V = (size_t)dims[0] * dims[1] * dims[2];
    DevMem coef, warped;
    if (grad_U) coef.alloc(ctx, 3 * V * sizeof(float));
    warped.alloc(ctx, V * sizeof(float));
    const int r = (window - 1) / 2;
    const SimTile tl = choose_sim_tile(ctx, dims, window, metric, sc.s);
    SimItem it{};
    it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
    it.zc = tl.zc;
    it.F = F;
    it.I = I;
    it.U = U;
    it.M = warped.as<float>();
    it.coef = grad_U ? coef.as<float>() : nullptr;
    it.gU = grad_U;
    it.inv_nr = 1.0 / ((double)(dims[0] - 2 * r) * (dims[1] - 2 * r) * (dims[2] - 2 * r));
    it.js = nullptr;
    it.sim_out = ctx->step_acc;
    const size_t off = sc.add(it);
    sc.upload();
    MUSTER_HIP(hipMemsetAsync(ctx->step_acc, 0, sizeof(double), sc.s));
    MUSTER_HIP(launch_warp((const SimItem*)(sc.dev() + off), 1,
                           point_tiles(dims[0], dims[1], dims[2]), sc.s));
    const int tiles = stat_tiles(dims[0], dims[1], dims[2], tl.zc, tl.shape);
    MUSTER_HIP(launch_sim_stats((const SimItem*)(sc.dev() + off), 1, tiles, window, metric,
                                tl.shape, sc.s));
    if (grad_U)
      MUSTER_HIP(launch_sim_grad((const SimItem*)(sc.dev() + off), 1, tiles, window, tl.shape,
                                 sc.s));
    MUSTER_HIP(hipMemcpyAsync(sim_host, ctx->step_acc, sizeof(double), hipMemcpyDeviceToHost, sc.s));
    MUSTER_HIP(hipStreamSynchronize(sc.s));
  });
}

muster_status muster_sim_noalloc(muster_ctx* h, void* stream, const int dims[3], int window,
                                 int metric, const float* F, const float* I, const float* U,
                                 double* sim_host, float* grad_U) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && F && I && U && sim_host, "NULL argument");
    NEED(window == 3 || window == 5 || window == 7, "window must be 3, 5 or 7");
    NEED(metric == MUSTER_METRIC_LNCC || metric == MUSTER_METRIC_SILNCC, "unknown metric");
    check_dims(dims, window);
    const size_t V = (size_t)dims[0] * dims[1] * dims[2];
    // sum | warped image | (coefficients), each part on a 256-byte boundary
    const size_t m_off = 256;
    const size_t c_off = m_off + ((V * sizeof(float) + 255) & ~(size_t)255);
    const size_t need = c_off + (grad_U ? 3 * V * sizeof(float) : 0);
    NEED(V <= NOALLOC_MAX_VOXELS && need <= NOALLOC_SCRATCH_BYTES,
         "%zu voxels exceed the %zu of the allocation-free scratch", V,
         (size_t)NOALLOC_MAX_VOXELS);
    NEED(ctx->noalloc_scratch, "no scratch on this device");
    std::lock_guard<std::mutex> lk(ctx->mu);
    StepCall sc{ctx, (hipStream_t)stream, {}};
    unsigned char* base = static_cast<unsigned char*>(ctx->noalloc_scratch);
    double* sum = reinterpret_cast<double*>(base);
    // the tiling the context already holds for this shape, never a new
    // autotuning run (that would allocate its scratch problem)
    SimTile tl;
    tl.shape = 0;
    tl.zc = std::min(32, dims[0]);
    if (ctx->tile_mode == MUSTER_TILES_FIXED) {
      tl = ctx->fixed_tile;
      tl.zc = std::min(tl.zc, dims[0]);
    } else if (ctx->tile_mode == MUSTER_TILES_AUTOTUNE) {
      std::lock_guard<std::mutex> tk(ctx->tune_mu);
      auto f = ctx->tuned.find(tune_key(dims, window, metric));
      if (f != ctx->tuned.end()) tl = f->second;
    }
    const int r = (window - 1) / 2;
    SimItem it{};
    it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
    it.zc = tl.zc;
    it.F = F;
    it.I = I;
    it.U = U;
    it.M = reinterpret_cast<float*>(base + m_off);
    it.coef = grad_U ? reinterpret_cast<float*>(base + c_off) : nullptr;
    it.gU = grad_U;
    it.inv_nr = 1.0 / ((double)(dims[0] - 2 * r) * (dims[1] - 2 * r) * (dims[2] - 2 * r));
    it.js = nullptr;
    it.sim_out = sum;
    const size_t off = sc.add(it);
    sc.upload();
    // the sum starts at zero: a fill kernel (two floats of zero bits)
    MUSTER_HIP(launch_fill(reinterpret_cast<float*>(sum), 2, 0.f, sc.s));
    MUSTER_HIP(launch_warp((const SimItem*)(sc.dev() + off), 1,
                           point_tiles(dims[0], dims[1], dims[2]), sc.s));
    const int tiles = stat_tiles(dims[0], dims[1], dims[2], tl.zc, tl.shape);
    MUSTER_HIP(launch_sim_stats((const SimItem*)(sc.dev() + off), 1, tiles, window, metric,
                                tl.shape, sc.s));
    if (grad_U)
      MUSTER_HIP(launch_sim_grad((const SimItem*)(sc.dev() + off), 1, tiles, window, tl.shape,
                                 sc.s));
    MUSTER_HIP(hipMemcpyAsync(sim_host, sum, sizeof(double), hipMemcpyDeviceToHost, sc.s));
    MUSTER_HIP(hipStreamSynchronize(sc.s));
  });
}

muster_status muster_adam(muster_ctx* h, void* stream, int64_t n, float* x, const float* g, float* m,
                          float* v, int t, float lr, float beta1, float beta2, float eps) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && x && g && m && v, "NULL argument");
    NEED(n >= 0 && t >= 1, "need n >= 0 and t >= 1");
    NEED(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f, "bad Adam constants");
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t s = (hipStream_t)stream;
    MUSTER_HIP(launch_adam_flat(n, x, g, m, v, t, lr, beta1, beta2, eps, s));
    MUSTER_HIP(hipStreamSynchronize(s));
  });
}

muster_status muster_reg(muster_ctx* h, void* stream, const int dims[3], const float* phi,
                         double* reg_host, float* grad) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && phi && reg_host, "NULL argument");
    check_dims(dims, 2);
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t s = (hipStream_t)stream;
    MUSTER_HIP(hipMemsetAsync(ctx->step_acc, 0, sizeof(double), s));
    MUSTER_HIP(launch_reg(GridDims{dims[0], dims[1], dims[2]}, phi, ctx->step_acc, grad, s));
    MUSTER_HIP(hipMemcpyAsync(reg_host, ctx->step_acc, sizeof(double), hipMemcpyDeviceToHost, s));
    MUSTER_HIP(hipStreamSynchronize(s));
  });
}

muster_status muster_pool2(muster_ctx* h, void* stream, const int dims[3], const float* src,
                           float* dst) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && src && dst, "NULL argument");
    check_dims(dims, 2);
    NEED(dims[0] % 2 == 0 && dims[1] % 2 == 0 && dims[2] % 2 == 0, "dims must be even");
    std::lock_guard<std::mutex> lk(ctx->mu);
    StepCall sc{ctx, (hipStream_t)stream, {}};
    PoolItem it{};
    it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
    it.src = src;
    it.dst = dst;
    const size_t off = sc.add(it);
    sc.upload();
    const size_t n = (size_t)(dims[0] / 2) * (dims[1] / 2) * (dims[2] / 2);
    MUSTER_HIP(launch_pool2((const PoolItem*)(sc.dev() + off), 1, elem_tiles(n), sc.s));
    MUSTER_HIP(hipStreamSynchronize(sc.s));
  });
}

muster_status muster_smooth(muster_ctx* h, void* stream, const int dims[3], float sigma,
                            const float* src, float* dst) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && src && dst, "NULL argument");
    NEED(src != dst, "src and dst must differ");
    check_dims(dims, 1);
    NEED(sigma > 0.f && sigma <= MAX_SMOOTH_SIGMA, "sigma must be in (0, 22]");
    NEED(dims[0] <= SMOOTH_MAX_DIM && dims[1] <= SMOOTH_MAX_DIM && dims[2] <= SMOOTH_MAX_DIM,
         "every dimension must be at most 4096");
    for (int a = 0; a < 3; ++a)
      NEED(smooth_radius(dims[a], sigma) <= MAX_SMOOTH_RADIUS,
           "sigma needs a kernel radius above 128 along an axis (whole lines up to 257 voxels "
           "at small sigma)");
    std::lock_guard<std::mutex> lk(ctx->mu);
    StepCall sc{ctx, (hipStream_t)stream, {}};
    const size_t V = (size_t)dims[0] * dims[1] * dims[2];
    DevMem t1, t2;
    t1.alloc(ctx, 3 * V * sizeof(float));
    t2.alloc(ctx, 3 * V * sizeof(float));
    const float* srcs[3] = {src, t1.as<float>(), t2.as<float>()};
    float* dsts[3] = {t1.as<float>(), t2.as<float>(), dst};
    size_t offs[3];
    int tiles[3], lds[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
      SmoothItem it{};
      tiles[a] = smooth_item_setup(it, dims, a, sigma, &lds[a]);
      it.src = srcs[a];
      it.dst = dsts[a];
      offs[a] = sc.add(it);
    }
    sc.upload();
    for (int a = 0; a < 3; ++a)
      MUSTER_HIP(launch_smooth((const SmoothItem*)(sc.dev() + offs[a]), 1, tiles[a], lds[a], sc.s));
    MUSTER_HIP(hipStreamSynchronize(sc.s));
  });
}

muster_status muster_upsample2(muster_ctx* h, void* stream, const int dims[3], const float* src,
                               float* dst) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && src && dst, "NULL argument");
    check_dims(dims, 2);
    NEED((uint64_t)dims[0] * dims[1] * dims[2] * 8 * 3 < (uint64_t)INT32_MAX, "volume too large");
    std::lock_guard<std::mutex> lk(ctx->mu);
    StepCall sc{ctx, (hipStream_t)stream, {}};
    UpItem it{};
    it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
    it.src = src;
    it.dst = dst;
    const size_t off = sc.add(it);
    sc.upload();
    MUSTER_HIP(launch_upsample2((const UpItem*)(sc.dev() + off), 1,
                                up_tiles(dims[0], dims[1], dims[2]), sc.s));
    MUSTER_HIP(hipStreamSynchronize(sc.s));
  });
}

muster_status muster_upsample2_adjoint(muster_ctx* h, void* stream, const int dims[3],
                                       const float* src, float* dst) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && src && dst, "NULL argument");
    check_dims(dims, 2);
    NEED((uint64_t)dims[0] * dims[1] * dims[2] * 8 * 3 < (uint64_t)INT32_MAX, "volume too large");
    std::lock_guard<std::mutex> lk(ctx->mu);
    StepCall sc{ctx, (hipStream_t)stream, {}};
    UpItem it{};
    it.D = dims[0]; it.H = dims[1]; it.W = dims[2];
    it.src = src;
    it.dst = dst;
    const size_t off = sc.add(it);
    sc.upload();
    MUSTER_HIP(launch_upsample2_adj((const UpItem*)(sc.dev() + off), 1,
                                    up_adj_tiles(dims[0], dims[1], dims[2]), sc.s));
    MUSTER_HIP(hipStreamSynchronize(sc.s));
  });
}

// ---- measurement ----------------------------------------------------------------

muster_status muster_jacobian_det(muster_ctx* h, void* stream, const int dims[3], const float* U,
                                  float* det) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && U && det, "NULL argument");
    check_dims(dims, 2);
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t s = (hipStream_t)stream;
    MUSTER_HIP(launch_jacobian_det(GridDims{dims[0], dims[1], dims[2]}, U, det, s));
    MUSTER_HIP(hipStreamSynchronize(s));
  });
}

muster_status muster_field_metrics(muster_ctx* h, void* stream, const int dims[3], const float* ref,
                                   const float* est, const unsigned char* roi, double* eu,
                                   double* pcc, double* slope) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && ref && est && eu && pcc && slope, "NULL argument");
    check_dims(dims, 1);
    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t s = (hipStream_t)stream;
    const int V = dims[0] * dims[1] * dims[2];
    double* acc = ctx->step_acc;  // 64 doubles
    MUSTER_HIP(hipMemsetAsync(acc, 0, 27 * sizeof(double), s));
    MUSTER_HIP(launch_field_stats(V, ref, est, roi, acc, s));
    double t[27];
    MUSTER_HIP(hipMemcpyAsync(t, acc, sizeof t, hipMemcpyDeviceToHost, s));
    MUSTER_HIP(hipStreamSynchronize(s));
    const double n = t[0];
    NEED(n > 0, "the region of interest is empty");
    *eu = t[1] / n;
    double ma[3], mb[3], Saa[3][3], Sba[3][3];
    for (int c = 0; c < 3; ++c) {
      ma[c] = t[2 + c] / n;
      mb[c] = t[5 + c] / n;
    }
    for (int c = 0; c < 3; ++c)
      for (int e = 0; e < 3; ++e) {
        Saa[c][e] = t[8 + 3 * c + e] - n * ma[c] * ma[e];
        Sba[c][e] = t[17 + 3 * c + e] - n * mb[c] * ma[e];
      }
    const double Sbb = t[26] - n * (mb[0] * mb[0] + mb[1] * mb[1] + mb[2] * mb[2]);
    const double tr_ba = Sba[0][0] + Sba[1][1] + Sba[2][2];
    const double tr_aa = Saa[0][0] + Saa[1][1] + Saa[2][2];
    *pcc = tr_ba / std::sqrt(tr_aa * Sbb);
    // A = Sba Saa^-1 (least squares of est on ref with an intercept); B = tr(A) / 3
    const double (&m)[3][3] = Saa;
    const double det = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
                       m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                       m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
    double inv[3][3];
    inv[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) / det;
    inv[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) / det;
    inv[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / det;
    inv[1][0] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) / det;
    inv[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / det;
    inv[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) / det;
    inv[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) / det;
    inv[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) / det;
    inv[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / det;
    double tr = 0.0;
    for (int c = 0; c < 3; ++c)
      for (int e = 0; e < 3; ++e) tr += Sba[c][e] * inv[e][c];
    *slope = tr / 3.0;
  });
}

muster_status muster_ctx_set_tiling(muster_ctx* h, int mode, int shape, int zchunk) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx, "NULL context");
    NEED(mode == MUSTER_TILES_DEFAULT || mode == MUSTER_TILES_AUTOTUNE || mode == MUSTER_TILES_FIXED,
         "unknown tiling mode %d", mode);
    if (mode == MUSTER_TILES_FIXED) {
      NEED(shape >= 0 && shape < SIM_SHAPES, "shape must be in 0..%d", SIM_SHAPES - 1);
      NEED(zchunk >= 1, "zchunk must be positive");
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tile_mode = mode;
    if (mode == MUSTER_TILES_FIXED) ctx->fixed_tile = SimTile{shape, zchunk};
  });
}

muster_status muster_ctx_sim_tiling(muster_ctx* h, void* stream, const int dims[3], int window,
                                    int metric, int* shape, int* zchunk) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx && shape && zchunk, "NULL argument");
    NEED(window == 3 || window == 5 || window == 7, "window must be 3, 5 or 7");
    NEED(metric == MUSTER_METRIC_LNCC || metric == MUSTER_METRIC_SILNCC, "unknown metric");
    check_dims(dims, window);
    std::lock_guard<std::mutex> lk(ctx->mu);
    const SimTile t = choose_sim_tile(ctx, dims, window, metric, (hipStream_t)stream);
    *shape = t.shape;
    *zchunk = t.zc;
  });
}

muster_status muster_ctx_memory(muster_ctx* h, uint64_t* in_use, uint64_t* peak, int reset_peak) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx, "ctx is NULL");
    if (in_use) *in_use = ctx->arena.used();
    if (peak) *peak = ctx->arena.peak();
    if (reset_peak) ctx->arena.reset_peak();
  });
}

muster_status muster_ctx_trim(muster_ctx* h, uint64_t* released) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx, "ctx is NULL");
    MUSTER_HIP(hipSetDevice(ctx->device));
    const uint64_t b = ctx->arena.trim();
    if (released) *released = b;
  });
}

muster_status muster_set_kernel_timing(muster_ctx* h, int enable) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx, "ctx is NULL");
    ctx->timing = enable != 0;
    ctx->timing_mask = enable != 0 ? (1u << MUSTER_K_COUNT) - 1u : 0u;
  });
}

muster_status muster_set_kernel_timing_mask(muster_ctx* h, uint32_t mask) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx, "ctx is NULL");
    NEED(mask < (1u << MUSTER_K_COUNT), "mask names a kernel class beyond MUSTER_K_COUNT");
    ctx->timing = mask != 0;
    ctx->timing_mask = mask;
  });
}

muster_status muster_kernel_stats(muster_ctx* h, int64_t launches[MUSTER_K_COUNT],
                                  double ms[MUSTER_K_COUNT], double bytes[MUSTER_K_COUNT]) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx, "ctx is NULL");
    resolve_timing(ctx);
    for (int k = 0; k < MUSTER_K_COUNT; ++k) {
      if (launches) launches[k] = ctx->stats.launches[k];
      if (ms) ms[k] = ctx->stats.ms[k];
      if (bytes) bytes[k] = ctx->stats.bytes[k];
    }
  });
}

muster_status muster_kernel_stats_reset(muster_ctx* h) {
  Ctx* ctx = C(h);
  return guard(ctx, [&] {
    NEED(ctx, "ctx is NULL");
    resolve_timing(ctx);
    ctx->stats = KernelStats{};
  });
}

const char* muster_kernel_name(int k) {
  static const char* names[MUSTER_K_COUNT] = {"exp_fwd", "compose_fwd", "sim_stats", "sim_grad",
                                              "compose_bwd", "exp_bwd", "adam", "finish",
                                              "pool2", "upsample2", "smooth", "upsample2_adj",
                                              "rigid", "warp", "unstage"};
  if (k < 0 || k >= MUSTER_K_COUNT) return "";
  return names[k];
}

}  // extern "C"
