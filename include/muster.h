/*
 * muster.h -- C ABI of the MI355X (gfx950) implementation of the MUSTER
 * per-iteration optimisation path (Multi-Session Temporal Registration,
 * arXiv 2412.14671).
 *
 * Problem (paper Sec. 2.1-2.2): a series of N 3-D images I_1..I_N of one
 * subject, acquired at times t_1 < ... < t_N on one regular grid, is
 * registered by optimising N-1 stationary velocity fields phi_{i,i+1}
 * (Sec. 2.3).  Exp(phi) by scaling and squaring (Alg. 1) gives the forward
 * consecutive deformation and Exp(-phi) its inverse; every ordered pair of
 * sessions is reached by composing consecutive deformations
 * (Eq. cum_deformation).  Every session is warped onto every other one and
 * scored by windowed LNCC (Eq. LNCC, sum_lncc) or SiLNCC (Eq. sim_loss);
 * the diffusion regulariser of Eq. reg_ss is added (Eq. reg_sum) and Adam with
 * a linear warm-up and cosine decay takes the step, inside a coarse-to-fine
 * pyramid (Sec. 2.7).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - dims[3] = {D, H, W}; volumes are float32, C order, x (W) fastest.
 *  - A vector field is float32 [3][D][H][W] (structure of arrays, components
 *    z, y, x), holding displacements u = Phi - Omega in voxels of its grid.
 *  - Image series: [N][D][H][W].  SVFs: [N-1][3][D][H][W], index i holds
 *    phi_{i,i+1} (0-based).  Pair fields: [N(N-1)][3][D][H][W]; pair
 *    (target i, source j), i != j, is at index i*(N-1) + (j < i ? j : j-1) and
 *    holds U[j->i] = Phi_ji^i - Omega, the field on grid i that pulls I_j onto
 *    I_i.
 *  - Sampling is trilinear with the sample position clamped to the grid
 *    (border padding); fields sampled off the grid take border values.
 *  - Every pointer argument named *_dev is a device pointer in the context's
 *    device memory (e.g. from torch), 4-byte aligned (256 recommended);
 *    *_host pointers are host memory.  The library never frees or keeps a
 *    caller buffer after a call returns, except that muster_submit's buffers
 *    must stay valid until the job reaches a terminal state.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on it; calls that return host values synchronise it.
 *  - Functions return muster_status.  On error the outputs are unspecified,
 *    no job state is left behind, and muster_last_error() holds a message
 *    for the calling thread.  MUSTER_E_DEVICE means a HIP error: the context
 *    is poisoned and every later call on it returns MUSTER_E_DEVICE.
 *  - No C++ exception crosses this interface.
 */
#ifndef MUSTER_H_
#define MUSTER_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum muster_status {
  MUSTER_OK = 0,
  MUSTER_E_INVALID = 1,    /* bad argument (shape, pointer, parameter)          */
  MUSTER_E_NOMEM = 2,      /* the context's HBM budget or the device is full     */
  MUSTER_E_DEVICE = 3,     /* HIP runtime error; the context is poisoned         */
  MUSTER_E_BUSY = 4,       /* serving queue full                                 */
  MUSTER_E_NONFINITE = 5,  /* the job's loss became NaN or infinite              */
  MUSTER_E_CANCELLED = 6,  /* the job was cancelled                              */
  MUSTER_E_INTERNAL = 7    /* a bug: please report with muster_last_error()      */
} muster_status;

enum { MUSTER_METRIC_LNCC = 0, MUSTER_METRIC_SILNCC = 1 };
enum { MUSTER_EXP_STORE = 0, MUSTER_EXP_RECOMPUTE = 1 };
#define MUSTER_MAX_LEVELS 6

typedef struct muster_ctx muster_ctx;
typedef struct muster_saved muster_saved;

/* Optimisation parameters (Sec. 2.3, 2.4, 2.6, 2.7).  Fill with
 * muster_params_default() and change what differs. */
typedef struct muster_params {
  int levels;                      /* pyramid levels L, 1..MUSTER_MAX_LEVELS     */
  int iters[MUSTER_MAX_LEVELS];    /* Adam steps per level, coarse to fine        */
  int K;                           /* squarings in Exp, 1..20 (Alg. 1)            */
  int window;                      /* odd window edge w, 3..7                     */
  int metric;                      /* MUSTER_METRIC_LNCC or _SILNCC               */
  float alpha_ss;                  /* weight of L_ss (Eq. reg_sum), >= 0          */
  float lr;                        /* peak Adam learning rate, voxels per step    */
  float warmup;                    /* warm-up fraction of each level, [0, 1]      */
  float beta1, beta2, eps;         /* Adam constants                              */
  int exp_mode;                    /* MUSTER_EXP_STORE or _RECOMPUTE: keep the K
                                      squaring fields for the backward pass, or
                                      recompute them from phi                     */
  int use_graph;                   /* 1: replay each level's iteration as a
                                      captured hipGraph; 0: eager launches        */
  float smooth_sigma;              /* Gaussian smoothing of the flow before Exp
                                      (Sec. 2.4, Appendix A): the transfer
                                      function exp(-sigma^2 |omega|^2 / 2) on the
                                      periodic grid, sigma in voxels of the
                                      finest level, halved per coarser level;
                                      0 = off; at most 22.  Its spatial taps
                                      must fit a radius of 128 on every line of
                                      every level (below sigma ~2 they span the
                                      whole line, so such lines are at most 257
                                      voxels); each dimension is at most 4096  */
  float alpha_l2;                  /* weight of L_L2 (second form of Eq. reg_ss):
                                      (1/(N-1)) sum_i mean_p |phi_i(p)|^2; 0 = off */
  float alpha_ts;                  /* weight of L_ts (Eq. reg_ts):
                                      (1/(N-2)) sum_k mean_p |phi_{k-1}/dt_{k-1}
                                      - phi_k/dt_k|^2 with dt_k = t_{k+1} - t_k;
                                      needs the acquisition times; 0 = off.
                                      Both act on the flow Exp integrates (the
                                      smoothed flow when smoothing is on)         */
  int flow_factor;                 /* 1: the flows live on the image grid; 2: on
                                      a grid twice as coarse (the paper's stage
                                      geometry, Sec. 2.7).  Exp and the
                                      compositions run on the flow grid; the pair
                                      fields are carried up to the image grid
                                      for the similarity.  dims must then be
                                      divisible by 2^levels; smooth_sigma is in
                                      voxels of the finest flow grid; svf_out
                                      and pairs_out stay on the image grid (the
                                      flows carried up, in image voxels), while
                                      svf_init and the autograd svf are on the
                                      flow grid.  0 is read as 1.              */
  int rigid;                       /* 1: a rigid adjustment (Euler angles about
                                      z, y, x and a translation, in voxels, about
                                      the grid centre) per session but the first,
                                      optimised with the flows; its displacement
                                      is added to every pair field that samples
                                      that session (Sec. 2.5).  Registration
                                      entry points only (not the autograd ones) */
  int deterministic;               /* 1: results that do not depend on the order
                                      of atomic adds, so a job gives bit-identical
                                      flows alone, batched or served: the adjoint
                                      scatters that add into shared fields with
                                      atomics add 64-bit fixed point at a scale
                                      set per job and launch (one more reduce-only
                                      pass of those kernels and a fold, and
                                      6(N-1) more int64 fields of the flow
                                      grid), and the window statistics use
                                      the default tiling instead of the
                                      autotuner's.  Registration entry points
                                      only.  The rigid adjustment's sums remain
                                      FP64 atomics.  0 = off                     */
} muster_params;

/* Per-job result summary. */
typedef struct muster_report {
  int status;                      /* muster_status of the job                    */
  int iterations;                  /* Adam steps taken over all levels            */
  double loss_first;               /* loss at the first step of the first level   */
  double loss_last;                /* loss at the last step of the finest level   */
  double seconds;                  /* wall time from start (or submission) to end */
  double queue_seconds;            /* serving only: submission to admission       */
  uint64_t footprint_bytes;        /* device bytes the job held                   */
  double step_seconds;             /* wall time of the optimisation steps alone:
                                      every level's iterations, each level's run
                                      bracketed by stream synchronisations (job
                                      set-up, pyramid and level changes and the
                                      final outputs excluded); shared by all jobs
                                      of a batch; 0 for served jobs              */
} muster_report;

/* One registration job for the batched and serving entry points. */
typedef struct muster_job {
  int N;                           /* sessions, >= 2                              */
  int dims[3];                     /* finest grid {D, H, W}                       */
  const float* images_dev;         /* [N][D][H][W]                                */
  const double* times_host;        /* [N], finite, strictly increasing            */
  const float* svf_init_dev;       /* optional [N-1][3] fields at the coarsest
                                      level; NULL starts from phi = 0              */
  float* svf_out_dev;              /* [N-1][3][D][H][W] result                    */
  float* pairs_out_dev;            /* optional [N(N-1)][3][D][H][W] result; with
                                      a rigid adjustment these are the total
                                      deformations (pair field + rigid part)      */
  muster_params params;
  float* rigid_out_dev;            /* optional [N-1][6] result with params.rigid:
                                      angles (z, y, x; radians) and translation
                                      (voxels) of sessions 1..N-1                 */
} muster_job;

/* ---- context -------------------------------------------------------------- */

/* Create a context on HIP device `device`.  hbm_budget bounds the device
 * bytes the context may hold for workspaces (0 = 80 % of the device memory
 * free at creation).  The server admits jobs while their footprints fit it.
 * The context owns its arena, internal streams, graphs and autotune cache. */
muster_status muster_ctx_create(int device, uint64_t hbm_budget, muster_ctx** out);
/* Destroy a context (waits for its work; stops its server thread). */
muster_status muster_ctx_destroy(muster_ctx* ctx);

/* Tiling of the window-statistics kernels (warp + moments + Sim, and their
 * adjoint; Sec. 2.6).  A block owns a tile of window centres of shape
 * 0 = 8 x 32, 1 = 16 x 32 or 2 = 8 x 64 (y x x) and marches through a chunk
 * of `zchunk` slices in z.  Modes:
 *   MUSTER_TILES_DEFAULT  shape 0, zchunk 32;
 *   MUSTER_TILES_AUTOTUNE (the default) the fastest of every shape and
 *                         zchunk in {16, 32, 64}, timed once per problem
 *                         shape (D, H, W, window, metric) on scratch data of
 *                         that shape, then cached in the context (and, when
 *                         the environment variable MUSTER_TUNE_CACHE names a
 *                         file, appended to it and read back by later
 *                         contexts);
 *   MUSTER_TILES_FIXED    the given shape and zchunk.
 * zchunk is capped at D.  Results do not depend on the tiling beyond float
 * rounding.  MUSTER_E_INVALID for an unknown mode, shape or zchunk < 1. */
#define MUSTER_TILES_DEFAULT 0
#define MUSTER_TILES_AUTOTUNE 1
#define MUSTER_TILES_FIXED 2
muster_status muster_ctx_set_tiling(muster_ctx* ctx, int mode, int shape, int zchunk);
/* The tiling the context uses for one problem shape (tuning it now, on
 * `stream`, if the mode is AUTOTUNE and it is not cached). */
muster_status muster_ctx_sim_tiling(muster_ctx* ctx, void* stream, const int dims[3], int window,
                                    int metric, int* shape, int* zchunk);
/* Device bytes the context's arena holds now (*in_use) and the most it has
 * held (*peak) since the context was created or the mark was last reset;
 * either pointer may be NULL.  reset_peak != 0 resets the mark to the bytes
 * in use, after reading it.  Counts workspaces only (the caller's buffers
 * are not the library's); used to compare the stored and recomputed
 * squaring steps of the Exp adjoint.  Workspaces that finished jobs release
 * are not counted here: the arena keeps them for later requests of the
 * same size (see muster_ctx_trim). */
muster_status muster_ctx_memory(muster_ctx* ctx, uint64_t* in_use, uint64_t* peak,
                                int reset_peak);
/* Return to the device the workspaces the context keeps for reuse.  The
 * arena keeps what finished jobs release, by size, so that repeated
 * registrations of similar jobs allocate nothing (a device allocation of
 * tens of GB takes seconds); the kept bytes count against hbm_budget, and
 * an allocation that fails first takes back what every context of the
 * process keeps, then tries once more.  Call this to give the memory to
 * other users of the device.  *released (may be NULL): bytes returned.
 * Workspaces released while work that uses them may still be in flight are
 * handed out again only after a device synchronisation, and returned with
 * the device free, which waits for that work. */
muster_status muster_ctx_trim(muster_ctx* ctx, uint64_t* released);
/* Thread-local text of the last error on this thread ("" if none). */
const char* muster_last_error(void);
/* Library version string. */
const char* muster_version(void);

/* Defaults (readings where the paper is silent): levels 1, iters {100}, K 7,
 * window 5, LNCC, alpha_ss 1, lr 0.1, warm-up 0.2 (Sec. 2.7), Adam
 * (0.9, 0.999, 1e-8), store mode, graphs on, no smoothing. */
muster_status muster_params_default(muster_params* p);

/* Device bytes a job of N sessions on grid dims needs under params
 * (workspaces only; the caller's images and outputs are not counted). */
muster_status muster_footprint(int N, const int dims[3], const muster_params* p,
                               uint64_t* bytes);

/* ---- whole registration (Sec. 2.2-2.7) ---------------------------------- */

/* Blocking single-subject registration: runs the pyramid of params and
 * writes the final SVFs and, if pairs_out_dev is not NULL, every pair field
 * Phi_ji^i - Omega computed from them.  times_host is validated (finite and
 * strictly increasing); the spatial-smoothness path does not use it.
 * Errors: E_INVALID for N < 2, a dimension smaller than the window or not
 * divisible by 2^(levels-1), an even window or one outside 3..7, K outside
 * 1..20, bad times, NULL images/svf_out; E_NOMEM; E_NONFINITE when the loss
 * diverges; E_DEVICE. */
muster_status muster_register(muster_ctx* ctx, void* stream, int N, const int dims[3],
                              const float* images_dev, const double* times_host,
                              const muster_params* params, float* svf_out_dev,
                              float* pairs_out_dev, muster_report* report);

/* Batched registration of n_jobs subjects with uneven N and grids: every
 * stage of one iteration runs as one launch over all jobs, and the iteration
 * is replayed from one captured hipGraph per level.  All jobs must share
 * levels, iters, K, window and metric; reports[n_jobs] receives per-job
 * results.  Each job's result matches muster_register on it alone. */
muster_status muster_register_batch(muster_ctx* ctx, void* stream, int n_jobs,
                                    const muster_job* jobs, muster_report* reports);

/* ---- serving: continuous batching ---------------------------------------- */

/* Start the context's server thread.  max_queue bounds waiting jobs.
 * The server admits a waiting job when its footprint fits the context's free
 * budget, then advances every resident job by one iteration per tick (one
 * batched launch sequence); jobs join and leave between ticks. */
muster_status muster_server_start(muster_ctx* ctx, int max_queue);
/* Submit a job (E_BUSY if the queue is full, E_NOMEM if its footprint
 * exceeds the context's whole budget, so that it could never be admitted);
 * the job's buffers must stay valid until it is terminal.  *ticket
 * identifies it. */
muster_status muster_submit(muster_ctx* ctx, const muster_job* job, uint64_t* ticket);
/* State of a job: 0 queued, 1 running, 2 done, 3 failed, 4 cancelled. */
muster_status muster_poll(muster_ctx* ctx, uint64_t ticket, int* state);
/* Block until the job is terminal; fills *report and returns its status.
 * The ticket is released. */
muster_status muster_wait(muster_ctx* ctx, uint64_t ticket, muster_report* report);
/* Cancel a queued or running job (it becomes terminal with E_CANCELLED). */
muster_status muster_cancel(muster_ctx* ctx, uint64_t ticket);
/* Server counters: resident jobs, queued jobs, device bytes in use. */
muster_status muster_server_stats(muster_ctx* ctx, int* resident, int* queued,
                                  uint64_t* bytes_in_use);

/* ---- differentiable loss (autograd) -------------------------------------- */

/* L(phi) at one grid: Sec. 2.2 loss with alpha_ss L_ss + alpha_l2 L_L2 +
 * alpha_ts L_ts (Eq. reg_sum), for images [N][D][H][W] and svf
 * [N-1][3][D][H][W] (K, window, metric, the alphas and smooth_sigma of params
 * are used).  times_host (N doubles, strictly increasing) is required when
 * alpha_ts > 0 and N >= 3, else it may be NULL.  Writes *loss_host
 * (synchronises the stream) and returns in *saved the state the backward pass
 * needs; the caller's buffers must stay valid until muster_saved_free. */
muster_status muster_loss_forward(muster_ctx* ctx, void* stream, int N, const int dims[3],
                                  const float* images_dev, const double* times_host,
                                  const float* svf_dev, const muster_params* params,
                                  double* loss_host, muster_saved** saved);
/* grad_svf_dev[N-1][3][D][H][W] = grad_out * dL/dphi by the hand-written
 * adjoints of every step.  The saved state can be used once. */
muster_status muster_loss_backward(muster_ctx* ctx, void* stream, muster_saved* saved,
                                   double grad_out, float* grad_svf_dev);
muster_status muster_saved_free(muster_saved* saved);

/* ---- single steps (for tests and tools) ---------------------------------- */

/* disp = Exp(sign * svf) - Omega by K squarings (Alg. 1, displacement form
 * u_{s+1} = u_s + u_s o (Omega + u_s), u_0 = sign*svf/2^K).  If steps_dev is
 * not NULL it receives u_1..u_K as [K][3][D][H][W]. */
muster_status muster_exp(muster_ctx* ctx, void* stream, const int dims[3], int K, int sign,
                         const float* svf_dev, float* disp_dev, float* steps_dev);
/* grad_svf = d<G, Exp(sign*svf)>/dsvf for G = grad_disp (adjoint of
 * muster_exp), in MUSTER_EXP_STORE or _RECOMPUTE mode.  With K >= 2 the
 * squaring steps hand their scatter boxes to each other through staging
 * slots, with the same kernels as the registration's backward pass;
 * mode | MUSTER_EXP_FLAT adds every step into a flat field instead. */
#define MUSTER_EXP_FLAT 4
muster_status muster_exp_bwd(muster_ctx* ctx, void* stream, const int dims[3], int K,
                             int sign, const float* svf_dev, const float* grad_disp_dev,
                             float* grad_svf_dev, int mode);
/* out = U_prev + C o (Omega + U_prev)  (Eq. cum_deformation). */
muster_status muster_compose(muster_ctx* ctx, void* stream, const int dims[3],
                             const float* U_prev_dev, const float* C_dev, float* out_dev);
/* Adjoint of muster_compose for G = dL/dout: ADDS dL/dU_prev to
 * G_prev_dev and dL/dC to G_C_dev (both must be initialised by the caller). */
muster_status muster_compose_bwd(muster_ctx* ctx, void* stream, const int dims[3],
                                 const float* U_prev_dev, const float* C_dev,
                                 const float* G_dev, float* G_prev_dev, float* G_C_dev);
/* Sim(F, I o (Omega + U)) for one pair (Eq. sum_lncc / sim_loss) into
 * *sim_host (synchronises); if grad_U_dev is not NULL it receives dSim/dU. */
muster_status muster_sim(muster_ctx* ctx, void* stream, const int dims[3], int window,
                         int metric, const float* F_dev, const float* I_dev,
                         const float* U_dev, double* sim_host, float* grad_U_dev);
/* muster_sim without allocating device memory, for callers that cannot
 * call hipMalloc: code under HIP graph capture, tight serving loops,
 * harnesses that forbid it.  The same kernels and arguments as muster_sim;
 * the warped image, the window coefficients and the sum live in a scratch
 * array of 96 MiB + 256 bytes that each GPU the library runs on holds from
 * the first context created on it until the process ends, so the grid is at
 * most 6 * 2^20 voxels (MUSTER_E_INVALID beyond).  The window statistics use
 * the context's fixed tiling, or the tiling it has already tuned for this
 * shape, else the default one (never a new autotuning run).  Every call on a
 * GPU shares that GPU's scratch: calls that overlap on one GPU (other
 * streams, threads or contexts) race and must be serialised by the caller.
 * Synchronises the stream. */
muster_status muster_sim_noalloc(muster_ctx* ctx, void* stream, const int dims[3], int window,
                                 int metric, const float* F_dev, const float* I_dev,
                                 const float* U_dev, double* sim_host, float* grad_U_dev);
/* One Adam step (PyTorch semantics, bias-corrected, step number t >= 1) on n
 * floats in place. */
muster_status muster_adam(muster_ctx* ctx, void* stream, int64_t n, float* x_dev,
                          const float* g_dev, float* m_dev, float* v_dev, int t, float lr,
                          float beta1, float beta2, float eps);
/* L_ss of one field (Eq. reg_ss, forward differences, mean per component and
 * axis) into *reg_host, and if grad_dev is not NULL its gradient. */
muster_status muster_reg(muster_ctx* ctx, void* stream, const int dims[3],
                         const float* phi_dev, double* reg_host, float* grad_dev);
/* 2x2x2 mean of a volume with even dims (one pyramid level down). */
muster_status muster_pool2(muster_ctx* ctx, void* stream, const int dims[3],
                           const float* src_dev, float* dst_dev);
/* Gaussian smoothing of a vector field [3][D][H][W] (Sec. 2.4, Appendix A):
 * the Fourier-domain filter exp(-sigma^2 |omega|^2 / 2) of the periodic grid
 * (omega in radians per voxel, sigma in voxels, 0 < sigma <= 22), applied as
 * one circular convolution per axis whose taps are that filter's inverse DFT
 * along the axis, kept out to where they sum below 2^-26 (the whole line at
 * small sigma); the radius must be at most 128 on every axis.  Each
 * dimension is at most 4096 (a whole line is staged on chip).  src and dst
 * must not overlap; MUSTER_E_INVALID otherwise. */
muster_status muster_smooth(muster_ctx* ctx, void* stream, const int dims[3], float sigma,
                            const float* src_dev, float* dst_dev);
/* Displacement field on the 2x finer grid: dst(x) = 2 * src((x - 0.5)/2);
 * dims are the coarse dims, dst is [3][2D][2H][2W]. */
muster_status muster_upsample2(muster_ctx* ctx, void* stream, const int dims[3],
                               const float* src_dev, float* dst_dev);
/* Adjoint of muster_upsample2 (how a gradient on the fine grid reaches the
 * coarse field; Sec. 2.7 with a flow grid coarser than the images): src is
 * [3][2D][2H][2W], dst [3][D][H][W] is overwritten; dims are the coarse dims. */
muster_status muster_upsample2_adjoint(muster_ctx* ctx, void* stream, const int dims[3],
                                       const float* src_dev, float* dst_dev);

/* ---- outputs and evaluation (Sec. 2.8) ------------------------------------ */

/* Jacobian determinant of Omega + U at every voxel: det(I + grad U), the
 * derivatives by central differences inside the grid and one-sided
 * differences at its faces.  U [3][D][H][W] in voxels, det [D][H][W].  Every
 * dimension must be at least 2. */
muster_status muster_jacobian_det(muster_ctx* ctx, void* stream, const int dims[3],
                                  const float* U_dev, float* det_dev);
/* Metrics of an estimated displacement field against a reference over a
 * region of interest (roi_dev: one byte per voxel, non-zero = inside; NULL =
 * every voxel): eu = mean |est - ref|; pcc = the vector Pearson correlation
 * (both fields centred by their mean vectors); slope = trace(A) / 3 for the
 * least-squares fit est = A ref + b.  Sums are accumulated in FP64.
 * MUSTER_E_INVALID for an empty region. */
muster_status muster_field_metrics(muster_ctx* ctx, void* stream, const int dims[3],
                                   const float* ref_dev, const float* est_dev,
                                   const unsigned char* roi_dev, double* eu, double* pcc,
                                   double* slope);

/* ---- measurement --------------------------------------------------------- */

enum {
  MUSTER_K_EXP_FWD = 0, MUSTER_K_COMPOSE_FWD, MUSTER_K_SIM_STATS, MUSTER_K_SIM_GRAD,
  MUSTER_K_COMPOSE_BWD, MUSTER_K_EXP_BWD, MUSTER_K_ADAM, MUSTER_K_FINISH,
  MUSTER_K_POOL, MUSTER_K_UPSAMPLE, MUSTER_K_SMOOTH, MUSTER_K_UPSAMPLE_ADJ, MUSTER_K_RIGID,
  MUSTER_K_WARP, MUSTER_K_UNSTAGE, MUSTER_K_COUNT
};
/* When enabled, eager launches (graphs off) of each kernel class are
 * bracketed by HIP events on the stream they run on. */
muster_status muster_set_kernel_timing(muster_ctx* ctx, int enable);
/* The same for the kernel classes whose bits are set in mask (bit k: class
 * k of the list above; 0 turns timing off).  Only those launches carry
 * events, so the others run as they do untimed; while any class is timed,
 * iterations launch eagerly instead of from a graph.  MUSTER_E_INVALID for
 * a bit at or beyond MUSTER_K_COUNT. */
muster_status muster_set_kernel_timing_mask(muster_ctx* ctx, uint32_t mask);
/* Per kernel class: launches, summed milliseconds and summed algorithmic
 * bytes (the unique bytes each launch must move) since the last reset. */
muster_status muster_kernel_stats(muster_ctx* ctx, int64_t launches[MUSTER_K_COUNT],
                                  double ms[MUSTER_K_COUNT], double bytes[MUSTER_K_COUNT]);
muster_status muster_kernel_stats_reset(muster_ctx* ctx);
const char* muster_kernel_name(int k);

#ifdef __cplusplus
}
#endif
#endif /* MUSTER_H_ */
