// Internal declarations shared by the HIP kernels and the host runtime.
//
// Every kernel takes a table of work items in device memory.  An item is one
// field-sized piece of work (one squaring of one direction, one composition,
// one session pair, ...) on its own grid, so a single launch can cover every
// interval, pair and subject of a batch with uneven grids.  Items in a table
// are sorted by tile0, the first global tile index of the item; a block finds
// its item by binary search.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace muster {

// Deterministic accumulation (a job's params.deterministic): every scatter
// that would add into a float field with global atomics adds 64-bit fixed
// point instead, at a scale shared by all blocks of the job in that launch:
// 2^(61 - e) with 2^e >= blocks * m, m the largest summed magnitude any of
// the job's blocks spreads (found by a pass of the same kernel that only
// reduces it), so no cell can overflow and integer adds make the sum
// independent of their order.  A fold then adds the fixed-point field into
// the float one.  One slot per such launch of an iteration.
constexpr int DET_SLOTS = 96;

// Per-job device state: optimiser step counter and schedule, loss
// accumulators and the loss history.  Lives in device memory so that a
// captured iteration can be replayed without host involvement.
struct JobState {
  int t;            // completed Adam steps at the current level
  int T;            // steps at this level
  int W;            // warm-up steps
  int nonfinite;    // set once the loss is not finite
  float lr0, b1, b2, eps;
  double loss_sim;  // accumulated over the current iteration
  double loss_reg;  // weighted regularisers
  double loss_ext;  // weighted L_L2 + L_ts of a loss-only forward pass
  double* history;  // loss per step (device), length hist_len
  int hist_len;
  int* flags;       // overflow flags of the staged Exp backward, cleared per iteration
  int n_flags;
  int hist_base;    // index of this level's first step in history
  unsigned int det_max[DET_SLOTS];  // deterministic mode: largest block magnitude (float bits)
};

struct GridDims {
  int D, H, W;
};

// u_{s+1} = u + u o (Omega + u) with u = a * src.
struct ExpFwdItem {
  int tile0;
  int D, H, W;
  const float* src;
  float* dst;
  float a;
  int pad;
};

// out = prev + C o (Omega + prev).
struct ComposeItem {
  int tile0;
  int D, H, W;
  const float* prev;
  const float* C;
  float* out;
};

// One backward squaring: given gin = dL/du_{s+1}, accumulate dL/du_s into
// gout (zeroed beforehand).  u_s = a * src.  If zero_in, gin is cleared
// after it is read.  If reg_w != 0, the regulariser gradient of src (= phi)
// times reg_w is added to the voxel's own term, and the regulariser value
// times reg_loss_w is added to the job's loss.
struct ExpBwdItem {
  int tile0;
  int D, H, W;
  const float* src;
  float* gin;
  float* gout;
  float a;
  int zero_in;
  float reg_w;       // weight of the L_ss gradient (0 = none)
  float reg_loss_w;  // weight of the L_ss value
  JobState* js;
  // L_L2 and L_ts at step 0 of a forward direction: the own term gains
  // w_self f_i + w_prev f_{i-1} + w_next f_{i+1} (flows of the neighbouring
  // intervals, NULL where absent), and the loss l2_loss_w |f_i|^2 +
  // ts_loss_w |f_{i-1} inv_dprev - f_i inv_dself|^2 per voxel.
  int ext;
  float w_self, w_prev, w_next;
  float l2_loss_w, ts_loss_w, inv_dprev, inv_dself;
  const float* flow_prev;
  const float* flow_next;
  // Staged accumulation between squaring steps.  A block that scatters
  // G_s with a box of bins that fits STAGE_CAP cells and stays within its
  // tile's 26 neighbours writes the box, plain, to its own slot of stage_out
  // ([tiles][3][STAGE_CAP]) and its extent to desc_out ([tiles][8]);
  // otherwise it adds into the flat gout with atomics, marks its descriptor
  // empty and sets *flag_out.  A step reading a staged G_{s+1} sums, at each
  // voxel, the boxes of its own tile and its neighbours that contain the
  // voxel, plus the flat gin where *flag_in is set (then clears it).
  const float* stage_in;
  const int* desc_in;
  const int* flag_in;
  float* stage_out;
  int* desc_out;
  int* flag_out;
  // Deterministic accumulation: where a block adds into gout with atomics it
  // adds into gout64 ([3][V] 64-bit fixed point) instead, at the scale of
  // the job's slot det_slot over det_blocks blocks (see DET_SLOTS); null
  // otherwise.
  long long* gout64;
  int det_slot;
  int det_blocks;
};

// Backward of one composition out = prev + C o (Omega + prev): given
// g = dL/dout, add (I + J_C^T) g to gprev (atomically if prev_atomic) and
// scatter g into gc.
struct ComposeBwdItem {
  int tile0;
  int D, H, W;
  const float* g;
  const float* prev;
  const float* C;
  float* gprev;
  float* gc;
  int prev_atomic;
  int pad;
  // Deterministic accumulation: the scatter into gc goes to gc64 ([3][V]
  // 64-bit fixed point) at the scale of the job's slot (see DET_SLOTS), and
  // gprev, whose only float writer in the launch is then this item, is
  // updated with plain stores; null otherwise.
  long long* gc64;
  JobState* js;
  int det_slot;
  int det_blocks;
};

// Fold of a 64-bit fixed-point field into its float field: f += q / scale,
// q = 0, over n = 3V elements, for the scale of the job's slot; skipped when
// flag is set and *flag is 0 (no block of the launch added into q).
struct DetFoldItem {
  int tile0;
  int n;
  float* f;
  long long* q;
  const JobState* js;
  const int* flag;
  int det_slot;
  int det_blocks;
};

// One session pair (target F = I_i, source I_j, field U = U[j->i]).
// Rigid adjustment of one session (Sec. 2.5): parameters (angles about z, y,
// x; translation), their Adam moments, the displacement the similarity
// kernels add, d(p) = A p + off with A = R - I and off = c + t - R c, and the
// gradient sums of the current iteration.
struct RigidState {
  float theta[3], t[3];
  float m[6], v[6];
  float A[9], off[3];
  double gsum[3];   // sum_p G(p)
  double gmom[9];   // sum_p G(p) (p - c)^T, row-major
};

// R = Rz Ry Rx in (z, y, x) components (Rz turns y towards x, Ry turns x
// towards z, Rx turns z towards y), or its derivative with respect to one
// angle (deriv = 0, 1, 2).
__host__ __device__ inline void rigid_rotation(const float th[3], int deriv, float R[9]) {
  float f[3][9];
  const int ax[3][2] = {{1, 2}, {2, 0}, {0, 1}};
  for (int k = 0; k < 3; ++k) {
    float c = cosf(th[k]), s = sinf(th[k]);
    const bool d = deriv == k;
    for (int e = 0; e < 9; ++e) f[k][e] = 0.f;
    if (d) {
      const float cc = -s;
      s = c;
      c = cc;
    } else {
      for (int e = 0; e < 3; ++e) f[k][4 * e] = 1.f;
    }
    const int a = ax[k][0], b = ax[k][1];
    f[k][3 * a + a] = c;
    f[k][3 * b + b] = c;
    f[k][3 * a + b] = -s;
    f[k][3 * b + a] = s;
  }
  float t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      float acc = 0.f;
      for (int l = 0; l < 3; ++l) acc += f[0][3 * i + l] * f[1][3 * l + j];
      t[3 * i + j] = acc;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      float acc = 0.f;
      for (int l = 0; l < 3; ++l) acc += t[3 * i + l] * f[2][3 * l + j];
      R[3 * i + j] = acc;
    }
}

struct SimItem {
  int tile0;
  int D, H, W;
  int zc;        // z-chunk length of this item's tiles
  int pad;
  const float* F;
  const float* I;
  const float* U;
  float* M;      // [V]: I warped by U (and the rigid adjustment), written by k_warp and read
                 // by k_sim_stats; may be the first plane of gU, which k_sim_grad overwrites
  float* coef;   // [3][V]: alpha, beta, gamma per window centre (may be null in sim_stats)
  float* gU;     // [3][V]: dSim/dU, written by sim_grad
  double inv_nr; // 1 / number of windows
  JobState* js;  // loss accumulator (may be null)
  double* sim_out;  // optional per-pair accumulator
  const RigidState* rigid;  // rigid adjustment of the source session, or null
};

// Gradient sums of a rigid adjustment from one pair's dSim/dU on the image grid.
struct RigidGradItem {
  int tile0;
  int D, H, W;
  const float* G;
  RigidState* rg;
};

// Adam step of one session's rigid parameters.
struct RigidStepItem {
  RigidState* rg;
  const JobState* js;
  float c[3];       // centre of the image grid
  float rot_lr;     // step scale of the angles (1 / largest half-extent)
};

// The gradient of one interval is g = scale * (g0f - g0b) (g0f, g0b are
// cleared after they are read), or gsrc when gsrc is set.  Mode 0: Adam step
// on phi.  Mode 1: gout = gscale * g.  Mode 2: gout = g (the combined
// gradient, for smoothing before the step).
struct AdamItem {
  int tile0;
  int n;          // voxels
  float* phi;
  float* g0f;     // dL/du_0 of the forward direction
  float* g0b;     // dL/du_0 of the backward direction
  const float* gsrc;
  float* m;
  float* v;
  float* gout;
  float scale;    // 2^-K
  float gscale;   // mode 1: grad_out
  int mode;
  int pad;
  JobState* js;
};

// The gradient of an SVF from the staged G_0 of its two directions:
// out = scale * (G_0 forward - G_0 backward), over point tiles.  Each
// direction's stage / desc / flag are those of its last backward squaring and
// gflat its flat overflow (cleared where read).
struct PullItem {
  int tile0;
  int D, H, W;
  const float* stage[2];
  const int* desc[2];
  const int* flag[2];
  float* gflat[2];
  float* out;
  float scale;
  // Diffusion regulariser of the interval's flow (Eq. reg_ss), when it is
  // added here rather than in the Exp backward's step 0: out gains
  // reg_w * dR/dflow, and the job's loss reg_loss_w * R(flow).
  float reg_w;
  float reg_loss_w;
  const float* flow;
  JobState* js;
};

// One separable pass of the periodic Gaussian smoothing along one axis, for
// one field of three components.  A tile holds whole lines of one component
// in LDS: `lines` adjacent x columns of lines along z or y, or `lines`
// consecutive rows along x.  Taps w[SMOOTH_WPAD + k] for k = 0..2*radius are
// the filter's weights at offsets k - radius along the periodic line (the
// host derives them from the Fourier-domain transfer function); every other
// entry is zero.
constexpr int MAX_SMOOTH_RADIUS = 128;
constexpr float MAX_SMOOTH_SIGMA = 22.0f;      // radius 5.66 sigma fits 128
constexpr int SMOOTH_S = 8;                    // outputs per thread along a line
constexpr int SMOOTH_WPAD = SMOOTH_S;
constexpr int SMOOTH_U = 8;                    // loads in flight per thread when staging
constexpr int SMOOTH_WLEN = 2 * MAX_SMOOTH_RADIUS + 1 + 2 * SMOOTH_WPAD;
constexpr int SMOOTH_LDS = 16384;              // floats of LDS per block, at most
constexpr int SMOOTH_LDS_TARGET = 8192;        // preferred, for occupancy
constexpr int SMOOTH_MAX_DIM = 4096;

struct SmoothItem {
  int tile0;
  int D, H, W;
  int axis;        // 0 = z, 1 = y, 2 = x
  int radius;
  int lines;       // lines per tile, a power of two in 1..64
  int lshift;      // log2(lines)
  int tiles_comp;  // tiles per component
  int pad[3];
  const float* src;
  float* dst;
  float w[SMOOTH_WLEN];
};

struct PoolItem {
  int tile0;
  int D, H, W;  // source dims
  const float* src;
  float* dst;
};

struct UpItem {
  int tile0;
  int D, H, W;  // coarse dims
  const float* src;
  float* dst;   // [3][2D][2H][2W]
};

// Tiles of the upsampling: UF_TZ x UF_TY x UF_TX fine voxels (D, H, W
// coarse).
constexpr int UF_TZ = 8, UF_TY = 8, UF_TX = 32;
inline int up_tiles(int D, int H, int W) {
  return ((2 * D + UF_TZ - 1) / UF_TZ) * ((2 * H + UF_TY - 1) / UF_TY) *
         ((2 * W + UF_TX - 1) / UF_TX);
}

// Tiles of the upsampling adjoint: UA_TZ x UA_TY x UA_TX coarse voxels.
constexpr int UA_TZ = 4, UA_TY = 8, UA_TX = 16;
inline int up_adj_tiles(int D, int H, int W) {
  return ((D + UA_TZ - 1) / UA_TZ) * ((H + UA_TY - 1) / UA_TY) * ((W + UA_TX - 1) / UA_TX);
}

// Tiles of the gather/scatter kernels.
constexpr int PT_Z = 8, PT_Y = 8, PT_X = 16;   // 1024 voxels, 256 threads
constexpr int PT_VOX = PT_Z * PT_Y * PT_X;
constexpr int BLOCK = 256;
constexpr int SCATTER_CELLS = 2048;          // LDS bins per component
constexpr int STAGE_CAP = SCATTER_CELLS;      // cells per component of a staging slot
// Tiles of the windowed-statistics kernels: TY x TX columns, z chunks.
// Tile shapes (centres in y x x) of the window-statistics kernels; the block
// has one thread per centre.
constexpr int SIM_SHAPES = 3;
constexpr int SIM_SHAPE_Y[SIM_SHAPES] = {8, 16, 8};
constexpr int SIM_SHAPE_X[SIM_SHAPES] = {32, 32, 64};
constexpr int ELEM_PER_BLOCK = 1024;           // elementwise kernels

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline int point_tiles(int D, int H, int W) {
  return ceil_div(D, PT_Z) * ceil_div(H, PT_Y) * ceil_div(W, PT_X);
}
inline int stat_tiles(int D, int H, int W, int zc, int shape) {
  return ceil_div(D, zc) * ceil_div(H, SIM_SHAPE_Y[shape]) * ceil_div(W, SIM_SHAPE_X[shape]);
}

// Launchers (kernels.hip).  All return hipError_t of the launch.
// Start and stop events for every following launch on this thread (null:
// untimed).  Each plan stage is one launch.
void set_launch_events(hipEvent_t start, hipEvent_t stop);
hipError_t launch_exp_fwd(const ExpFwdItem* items, int n_items, int n_tiles, hipStream_t s);
hipError_t launch_compose_fwd(const ComposeItem* items, int n_items, int n_tiles, hipStream_t s);
// staged: 0 flat in / flat out, 1 flat in / staged out, 2 staged in / staged out,
// 3 staged in / flat out
// reg: some item adds the regulariser terms (reg_w != 0 or ext); without it
// a leaner variant of the kernel runs.
hipError_t launch_exp_bwd(const ExpBwdItem* items, int n_items, int n_tiles, int staged, bool reg,
                          hipStream_t s);
// A staged G_0 (stage_in, desc_in, flag_in of each item) to the flat gout.
hipError_t launch_unstage(const ExpBwdItem* items, int n_items, int n_tiles, hipStream_t s);
hipError_t launch_pull_combine(const PullItem* items, int n_items, int n_tiles, hipStream_t s);
hipError_t launch_compose_bwd(const ComposeBwdItem* items, int n_items, int n_tiles,
                              hipStream_t s);
// Deterministic mode: the passes of the composition and Exp adjoints that
// only reduce each job's largest block magnitude into its slot (no other
// writes), the fold of the fixed-point fields, and the clearing of the slots.
hipError_t launch_compose_bwd_detmax(const ComposeBwdItem* items, int n_items, int n_tiles,
                                     hipStream_t s);
hipError_t launch_exp_bwd_detmax(const ExpBwdItem* items, int n_items, int n_tiles, int staged,
                                 hipStream_t s);
hipError_t launch_det_fold(const DetFoldItem* items, int n_items, int n_tiles, hipStream_t s);
hipError_t launch_det_clear(JobState* const* states, int n_jobs, hipStream_t s);
// M = I o (Omega + U) of each item, over point tiles of its grid.
hipError_t launch_warp(const SimItem* items, int n_items, int n_tiles, hipStream_t s);
hipError_t launch_sim_stats(const SimItem* items, int n_items, int n_tiles, int window, int metric,
                            int shape, hipStream_t s);
hipError_t launch_sim_grad(const SimItem* items, int n_items, int n_tiles, int window, int shape,
                           hipStream_t s);
hipError_t launch_adam(const AdamItem* items, int n_items, int n_tiles, hipStream_t s);
hipError_t launch_smooth(const SmoothItem* items, int n_items, int n_tiles, int lds_floats,
                         hipStream_t s);
// Fills the geometry and taps of a smoothing item; returns its tile count and
// raises *lds_floats to the LDS the item needs.
int smooth_item_setup(SmoothItem& it, const int dims[3], int axis, float sigma, int* lds_floats);
// Radius of the smoothing taps on a periodic line of n samples.
int smooth_radius(int n, float sigma);
hipError_t launch_finish(JobState* const* states, int n_jobs, hipStream_t s);
hipError_t launch_pool2(const PoolItem* items, int n_items, int n_tiles, hipStream_t s);
hipError_t launch_upsample2(const UpItem* items, int n_items, int n_tiles, hipStream_t s);
// adjoint: src [3][2D][2H][2W] (fine), dst [3][D][H][W] (coarse), tiles over the coarse grid
hipError_t launch_upsample2_adj(const UpItem* items, int n_items, int n_tiles, hipStream_t s);
hipError_t launch_adam_flat(int64_t n, float* x, const float* g, float* m, float* v, int t,
                            float lr, float b1, float b2, float eps, hipStream_t s);
hipError_t launch_reg(GridDims d, const float* phi, double* out, float* grad, hipStream_t s);
// out += l2w sum_p |f(p)|^2 + tsw sum_p |fprev(p) inv_dp - f(p) inv_ds|^2 (fprev may be NULL)
hipError_t launch_reg_ext(GridDims d, const float* f, const float* fprev, float l2w, float tsw,
                          float inv_dp, float inv_ds, double* out, hipStream_t s);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s);

// Scratch of the allocation-free similarity entry point: a file-scope device
// array (each GPU holds its own copy until the process ends) with the pair's
// sum in its first 256 bytes, then the warped source image and the window
// coefficients, for grids of up to NOALLOC_MAX_VOXELS voxels.
constexpr size_t NOALLOC_MAX_VOXELS = (size_t)6 << 20;
constexpr size_t NOALLOC_SCRATCH_BYTES = 256 + 16 * NOALLOC_MAX_VOXELS;
// Device address of the scratch array on `device`, which must be current:
// looked up once per device with hipGetSymbolAddress and kept (the array's
// name is a host-side stand-in, not a device address).
hipError_t noalloc_scratch_address(int device, void** ptr);
hipError_t launch_jacobian_det(GridDims d, const float* U, float* out, hipStream_t s);
hipError_t launch_rigid_grad(const RigidGradItem* items, int n_items, int n_tiles, hipStream_t s);
hipError_t launch_rigid_step(const RigidStepItem* items, int n_items, hipStream_t s);
// field [3][D][H][W] += the displacement of a rigid state
hipError_t launch_add_rigid(GridDims d, float* field, const RigidState* rg, hipStream_t s);
// 27 sums over the voxels with roi[p] != 0 (all if roi is NULL), added to out
hipError_t launch_field_stats(int V, const float* a, const float* b, const unsigned char* roi,
                              double* out, hipStream_t s);
// p[c][z][y][x] = off + amp * (a smooth periodic pattern); scratch data for
// the autotuner.
hipError_t launch_pattern(float* p, int64_t n, const int dims[3], float off, float amp,
                          float phase, hipStream_t s);

}  // namespace muster
