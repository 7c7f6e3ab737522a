/*
 * nbody.h - C ABI of libnbody.so: direct-sum softened gravity on AMD MI355X (gfx950).
 *
 * The library evaluates, for every i-particle,
 *     a_i   =  sum_{j != i} m_j (x_j - x_i) / (|x_j - x_i|^2 + eps^2)^{3/2}
 *     phi_i = -sum_{j != i} m_j / (|x_j - x_i|^2 + eps^2)^{1/2}
 * (Hamada & Iitaka, Sec. 1.1, eq. (1); the potential is the quantity accumulated by
 * the force-jerk-potential pipeline of Appendix A), with G = 1.  Pair arithmetic is
 * FP32; accumulation is plain FP32, FP32 with FP64 per-tile reduction, or FP32
 * with two-sum compensation (Sec. 2.2.2, eq. (2) is the paper's two-level form);
 * the per-particle reduction of partial sums and the outputs are FP64.
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller.  Positions are
 *     structure-of-arrays: pos[0..n) holds x, pos[n..2n) y, pos[2n..3n) z ("[3][n]").
 *     acc and grad_pos use the same [3][n] layout.  Arrays must be 4-byte aligned
 *     (float) or 8-byte aligned (double).
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Every call
 *     only enqueues work on it and returns without synchronising, except where a
 *     function says otherwise.
 *   - Outputs must not alias inputs.  n = 0 is a valid no-op.
 *   - eps must be finite and > 0 (the self pair would otherwise be 0/0).
 *   - NaN or Inf in the inputs propagate to the outputs; they are not checked.
 *   - Scratch memory: if opts->workspace is NULL the library uses a per-device
 *     buffer it allocates and grows on demand (calls on several streams of one
 *     device that overlap in time then race; give each stream its own workspace).
 *     A call on a stream that is being captured into a HIP graph must pass
 *     opts->workspace (at least the nbody_workspace_size* bytes of that call, kept
 *     alive as long as the graph): with a NULL workspace it returns NBODY_ECAPTURE
 *     and enqueues nothing, since a later call may reallocate the library's buffer
 *     under the recorded graph.  A too small workspace returns NBODY_EINVAL.
 *   - Errors: a negative status; nbody_last_error() returns a message for the
 *     calling thread.  Invalid arguments are detected before anything is enqueued.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define NBODY_API __attribute__((visibility("default")))
#else
#define NBODY_API
#endif

typedef int32_t nbody_status;
#define NBODY_OK 0
#define NBODY_EINVAL (-1)      /* bad size, NULL pointer, eps, offsets or option   */
#define NBODY_ENOMEM (-2)      /* device allocation failed                         */
#define NBODY_EHIP (-3)        /* HIP runtime error (message has the HIP text)     */
#define NBODY_ECAPTURE (-4)    /* stream is capturing and no workspace was given    */
#define NBODY_EUNSUPPORTED (-5)/* option combination not built                     */

/* Accumulation of the pair terms of one i-particle (Sec. 2.2.2 and Sec. 3.4). */
#define NBODY_PLAIN 0   /* one FP32 accumulator per j-segment; segments summed in FP32
                           (the paper's direct order with one segment, its FORCE-LOOP
                           of eq. (2) with 512-j segments)                              */
#define NBODY_FP64RED 1 /* FP32 partial over each block of j, added into FP64 registers
                           (the FORCE-LOOP of eq. (2) with an FP64 force memory)        */
#define NBODY_COMP 2    /* FP32 partial over each block of j, added into an FP32
                           (hi, lo) pair by an error-free two-sum; default              */

/* Reference centre for FP64 positions (every *_f64 entry point, the leapfrog, its
 * adjoint and the Hermite integrator). */
#define NBODY_CENTRE_NONE 0   /* pair arithmetic on fp32(x)                              */
#define NBODY_CENTRE_SYSTEM 1 /* on fp32(x - c), c = FP64 mean position of the system;
                                 default                                                 */
#define NBODY_CENTRE_TILE 2   /* on fp32(x - c_I), c_I = FP64 mean of the i-tile (256 x
                                 ipl consecutive particles), j's converted for each i-tile
                                 as they are staged; pays off when consecutive particles
                                 are spatially close (see nbody_morton_order).  Batched
                                 plans return NBODY_EUNSUPPORTED.                        */

typedef struct nbody_opts {
    int32_t precision;  /* NBODY_PLAIN, NBODY_FP64RED or NBODY_COMP                   */
    int32_t centre;     /* NBODY_CENTRE_*; ignored by the FP32-position entry points  */
    int32_t self_pot;   /* 0: phi excludes j == i (default); 1: phi includes -m_i/eps */
    int32_t ipl;        /* i-particles per lane: 1, 2, 4, 8; 0 = tuned/default        */
    int32_t jtile;      /* j-particles per LDS tile: 64, 128, 256, 512; 0 = default   */
    int32_t nseg;       /* j-segments per i-tile (grid y), <= 1024; 0 = chosen from n */
    int32_t jlanes;     /* lanes that share one i-particle's j-range (see below)       */
    int32_t symmetric;  /* 0: tuned; 1: off; 2: each unordered pair once (see below)   */
    void *workspace;    /* device scratch, or NULL for the library's per-device cache */
    size_t workspace_bytes;
} nbody_opts;

/* Launch shapes.  Three pair engines evaluate the same sums:
 *   - the grid engine (jlanes = 1): a block of 256 lanes holds 256 * ipl i-particles
 *     and walks one of nseg j-segments in LDS tiles of jtile records (64 to 512);
 *     the segment partial sums go to scratch memory and a second kernel adds them
 *     per particle in FP64 (the paper's i-parallel FORCE-LOOP, Sec. 2.2);
 *   - the split engine (jlanes = 8, 16, 32 or 64; ipl = 1 or 2; jtile = 256, 512,
 *     1024, or 2048 with jlanes >= 32; the adjoint: 256 or 512; nseg must be 0): for
 *     systems too small to
 *     fill the chip with whole i-tiles, the j-range of each i-particle is split over
 *     jlanes lanes of one wavefront, whose partial sums are added across the lanes
 *     in FP64 (PLAIN: FP32) by DPP / permlane moves in a fixed order.  One launch, no
 *     scratch for partial sums.  Available for nbody_force, nbody_force_ex,
 *     nbody_force_f64, the leapfrog, nbody_force_vjp(_f64) and the leapfrog adjoint,
 *     not with NBODY_CENTRE_TILE (which uses the grid engine's i-tiles);
 *   - the symmetric engine (symmetric = 2; ipl = 1, 2 or 4; jtile = 64 or 128;
 *     jlanes 0 or 1): the pair term of eq. (1) is antisymmetric, so each unordered
 *     pair {i, j} is evaluated once and its term added to both particles.  Block rows
 *     of 512 * ipl particles take the pairs with every later particle, in work items
 *     of a few j-tiles (nseg: items in the longest row, 0 = chosen from n); the i-side
 *     sums are accumulated as in the grid engine, the j-side sums per wavefront (FP32,
 *     64 * ipl terms) and over the block's 8 wavefronts in FP64 (PLAIN: FP32), and a
 *     second kernel adds both per particle in a fixed order.  Scratch grows as
 *     n^2 / (256 * ipl) FP64 values (PLAIN: FP32).  Available for nbody_force,
 *     nbody_force_ex, nbody_force_f64 and the leapfrog, not with NBODY_CENTRE_TILE.  On
 *     MI355X it runs about as fast as the grid engine (the lane-to-lane moves of the
 *     j-side sums cost what the halved pair work saves), so it is never chosen by
 *     default.
 * jlanes = 0 and symmetric = 0 with ipl, jtile and nseg all 0 take the shape from the
 * tuning table (any engine); with any of them set the grid engine is used unless
 * jlanes > 1 or symmetric = 2 selects another.  Results are bitwise reproducible for
 * a given shape; different shapes round differently. */

/* Fills *opts with the defaults (NBODY_COMP, NBODY_CENTRE_SYSTEM, self excluded,
 * tile shape from the tuning table, library workspace). */
NBODY_API void nbody_opts_default(nbody_opts *opts);

/* Message of the last error on the calling thread ("" if none).  The pointer stays
 * valid until the next library call on this thread. */
NBODY_API const char *nbody_last_error(void);

/* Library version string. */
NBODY_API const char *nbody_version(void);

/* Bytes of scratch that nbody_force, nbody_force_ex, nbody_force_f64 and
 * nbody_leapfrog need for n particles with these options (0 for n <= 0 or invalid
 * options; the batched plan owns its own). */
NBODY_API size_t nbody_workspace_size(int64_t n, const nbody_opts *opts);

/* ------------------------------------------------------------------------------
 * Forces and potentials, all i against all j of one system (eq. (1)).
 *   n     particles, 0 <= n < 2^30
 *   pos   float [3][n], positions (read)
 *   mass  float [n], masses (read; any sign, zero allowed)
 *   eps   softening length (> 0); the kernel uses fp32(eps * eps)
 *   acc   double [3][n], accelerations (written)
 *   pot   double [n] potentials (written), or NULL to skip them
 * nbody_force uses the default options.  The j == i pair is left out of every sum
 * (the pair kernel hands it a massless copy of the particle, which adds exactly
 * zero); with opts->self_pot = 1 the FP64 reduction adds -m_i/eps, formed in FP64,
 * to phi.
 * ---------------------------------------------------------------------------- */
NBODY_API nbody_status nbody_force(int64_t n, const float *pos, const float *mass, float eps,
                         double *acc, double *pot, void *stream);
NBODY_API nbody_status nbody_force_ex(int64_t n, const float *pos, const float *mass, float eps,
                            double *acc, double *pot, const nbody_opts *opts, void *stream);

/* As nbody_force_ex, with FP64 positions pos64 double [3][n].  The pair arithmetic
 * stays FP32, on positions taken relative to the reference centre opts->centre
 * (computed on the device in FP64).  This is the entry point for integrator state
 * and for systems far from the origin. */
NBODY_API nbody_status nbody_force_f64(int64_t n, const double *pos64, const float *mass, float eps,
                             double *acc, double *pot, const nbody_opts *opts, void *stream);

/* ------------------------------------------------------------------------------
 * As nbody_force_ex, for callers that cannot allocate device memory: code being
 * captured into a HIP graph without a workspace of its own, tight serving loops,
 * harnesses that forbid hipMalloc.  It calls no hipMalloc, hipFree or allocating
 * library routine.  The grid engine's segment partial sums go to a static device
 * array of NBODY_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds until
 * the process ends; the split engine needs none, the symmetric engine's j-side sums
 * share it.  If the partial sums of the chosen shape do not fit, a tuned symmetric
 * shape gives way to the grid engine and fewer j-segments are used (unless
 * opts->symmetric is 2 or opts->nseg is set); a size or shape whose partial sums exceed the
 * array even then returns NBODY_EINVAL with the bytes it would need.  opts->workspace must be NULL.  All calls on one GPU share its
 * array: calls that overlap in time on one GPU (several streams, several host
 * threads) race and give wrong results; calls on one stream are ordered and safe.
 * Nothing in the array needs clearing between calls (every partial sum is written
 * before it is read).  Other arguments, results and errors as nbody_force_ex.
 * ---------------------------------------------------------------------------- */
#define NBODY_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20) /* 64 MiB per GPU */
NBODY_API nbody_status nbody_force_noalloc(int64_t n, const float *pos, const float *mass,
                                           float eps, double *acc, double *pot,
                                           const nbody_opts *opts, void *stream);

/* ------------------------------------------------------------------------------
 * Forces and potentials on one set of particles from another (the paper's library
 * call takes separate i- and j-arrays, Sec. 3.1; its driver keeps eps^2 per
 * i-particle, Appendix A).  Every (i, j) pair is summed: no pair is treated as a
 * self pair, so an i-particle that coincides with a j-particle gets 0 acceleration
 * and -m_j/eps_i potential from it (NaN if eps_i = 0).  Uses: an i-range of a
 * system against all of it (one GPU's shard of a larger system), interaction lists.
 *   ni      i-particles, 0 <= ni < 2^30; pos_i float [3][ni] (read)
 *   eps_i   float [ni] per-i softening lengths (read; each finite and >= 0, not
 *           checked), or NULL: eps for every i
 *   nj      j-particles, 0 <= nj < 2^30; pos_j float [3][nj], mass_j float [nj] (read)
 *   eps     uniform softening (finite, >= 0; eps^2 zero or a normal float)
 *   acc     double [3][ni] (written); pot double [ni] or NULL (written)
 *   opts    precision, ipl, jtile, nseg and workspace apply; centre and self_pot are
 *           ignored (the inputs are FP32 already); NULL = defaults
 * nj = 0 writes zeros.  Outputs must not alias inputs.  Scratch:
 * nbody_workspace_size_ij bytes (the per-device cache when opts->workspace is NULL).
 * ---------------------------------------------------------------------------- */
NBODY_API nbody_status nbody_force_ij(int64_t ni, const float *pos_i, const float *eps_i,
                                      int64_t nj, const float *pos_j, const float *mass_j,
                                      float eps, double *acc, double *pot,
                                      const nbody_opts *opts, void *stream);
NBODY_API size_t nbody_workspace_size_ij(int64_t ni, int64_t nj, const nbody_opts *opts);

/* ------------------------------------------------------------------------------
 * Force, jerk and potential in one pass: the force-jerk-potential pipeline of the
 * paper's Appendix A, the interaction a fourth-order Hermite integrator needs
 * (Sec. 4.1).  With d = x_j - x_i, w = v_j - v_i, s^2 = |d|^2 + eps^2:
 *   a_i = sum m_j d / s^3,  jerk_i = sum m_j (w / s^3 - 3 (d.w) d / s^5),
 *   phi_i = -sum m_j / s,
 * all i against all j of one system, j == i left out as in nbody_force (self_pot = 1
 * adds -m_i/eps to phi).
 *   n      particles, 0 <= n < 2^30
 *   pos    float [3][n], vel float [3][n], mass float [n] (read)
 *   eps    softening length (> 0, eps^2 a normal float)
 *   acc    double [3][n], jerk double [3][n] (written); pot double [n] or NULL
 *   opts   precision, self_pot, ipl, jtile, nseg, workspace; NULL = defaults
 * Scratch: nbody_workspace_size_jerk bytes (covers both entry points), from
 * opts->workspace or the per-device cache.  Outputs must not alias inputs.
 * ---------------------------------------------------------------------------- */
NBODY_API nbody_status nbody_force_jerk(int64_t n, const float *pos, const float *vel,
                                        const float *mass, float eps, double *acc, double *jerk,
                                        double *pot, const nbody_opts *opts, void *stream);
/* As nbody_force_jerk with FP64 state pos64, vel64 double [3][n]: the pair arithmetic
 * is FP32 on positions relative to the FP64 mean position and velocities relative to
 * the FP64 mean velocity of the system (opts->centre = NBODY_CENTRE_SYSTEM, default) or
 * of each i-tile (NBODY_CENTRE_TILE: pays off when consecutive particles are close in
 * phase space, e.g. after nbody_morton_order), or on the plain FP32 roundings
 * (NBODY_CENTRE_NONE). */
NBODY_API nbody_status nbody_force_jerk_f64(int64_t n, const double *pos64, const double *vel64,
                                            const float *mass, float eps, double *acc,
                                            double *jerk, double *pot, const nbody_opts *opts,
                                            void *stream);

/* ------------------------------------------------------------------------------
 * Force, jerk and potential on one set of particles from another: the force-jerk-
 * potential pipeline (Appendix A) behind the paper's separate i- and j-set library
 * call (Sec. 3.1).  A Hermite code with individual time steps evaluates only its
 * active particles this way, against the predicted state of all of them.  Every
 * (i, j) pair is summed with the formulas of nbody_force_jerk and one softening for
 * all: no pair is a self pair, so an i-particle that coincides with a j-particle gets
 * zero acceleration and jerk and -m_j/eps potential from it (NaN if eps = 0).
 *   ni      i-particles, 0 <= ni < 2^30; pos_i, vel_i float [3][ni] (read)
 *   nj      j-particles, 0 <= nj < 2^30; pos_j, vel_j float [3][nj], mass_j float [nj]
 *           (read)
 *   eps     softening (finite, >= 0; eps^2 zero or a normal float).  Coordinates must
 *           stay well below 1e18 in magnitude (unused slots of a j-tile sit there).
 *   acc     double [3][ni], jerk double [3][ni] (written); pot double [ni] or NULL
 *   opts    precision, ipl, jtile, nseg and workspace apply; centre and self_pot are
 *           ignored; NULL = defaults
 * nj = 0 writes zeros.  Outputs must not alias inputs.  Scratch:
 * nbody_workspace_size_jerk_ij bytes (the per-device cache when opts->workspace is NULL).
 * ---------------------------------------------------------------------------- */
NBODY_API nbody_status nbody_force_jerk_ij(int64_t ni, const float *pos_i, const float *vel_i,
                                           int64_t nj, const float *pos_j, const float *vel_j,
                                           const float *mass_j, float eps, double *acc,
                                           double *jerk, double *pot, const nbody_opts *opts,
                                           void *stream);
NBODY_API size_t nbody_workspace_size_jerk_ij(int64_t ni, int64_t nj, const nbody_opts *opts);
NBODY_API size_t nbody_workspace_size_jerk(int64_t n, const nbody_opts *opts);

/* Morton (Z-order) permutation of FP64 positions pos64 double [3][n]: perm int32 [n]
 * (device, written) lists the particle indices in order along the Z-curve of the
 * FP64 bounding box (ties broken by index).  Gathering the particles in this order
 * makes i-tiles spatially compact, which is what NBODY_CENTRE_TILE needs.  Uses the
 * library workspace (allocates outside capture). */
NBODY_API nbody_status nbody_morton_order(int64_t n, const double *pos64, int32_t *perm,
                                          void *stream);

/* ------------------------------------------------------------------------------
 * Kick-drift-kick leapfrog on FP64 state (the paper has no integrator; this is the
 * standard second-order symplectic scheme).  One step:
 *     v += (dt/2) a(x);   x += dt v;   a = a(x);   v += (dt/2) a
 * with a(x) from nbody_force_f64 (same options; opts->centre applies).
 *   pos64, vel64  double [3][n], updated in place
 *   acc           double [3][n]: on entry a(pos64) unless flags has
 *                 NBODY_LF_INIT_ACC (then it is computed first); on exit a(final pos)
 *   pot           double [n] potentials at the final positions, or NULL
 *   traj          double [nsteps+1][3][n] position checkpoints x_0 .. x_nsteps, or
 *                 NULL (these are the states the adjoint needs)
 *   nsteps >= 0, dt finite (negative dt integrates backwards).
 * ---------------------------------------------------------------------------- */
#define NBODY_LF_INIT_ACC 1
NBODY_API nbody_status nbody_leapfrog(int64_t n, double *pos64, double *vel64, const float *mass,
                                      float eps, double dt, int32_t nsteps, double *acc,
                                      double *pot, double *traj, int32_t flags,
                                      const nbody_opts *opts, void *stream);

/* HIP graph of nsteps leapfrog steps (as nbody_leapfrog without NBODY_LF_INIT_ACC and
 * without checkpoints) on fixed arrays: every nbody_graph_launch replays the steps on
 * the device with no host work per kernel.  The graph owns its own scratch memory
 * (allocated here, outside any capture); the arrays passed here must stay valid for
 * the graph's lifetime.  nbody_graph_destroy waits for the device first. */
typedef struct nbody_graph nbody_graph;
NBODY_API nbody_status nbody_graph_create_leapfrog(int64_t n, double *pos64, double *vel64,
                                                   const float *mass, float eps, double dt,
                                                   int32_t nsteps, double *acc, double *pot,
                                                   const nbody_opts *opts, void *stream,
                                                   nbody_graph **out);
NBODY_API nbody_status nbody_graph_launch(nbody_graph *graph, void *stream);
NBODY_API void nbody_graph_destroy(nbody_graph *graph);

/* Fourth-order Hermite integration with a shared step (the integrator the force-jerk
 * interaction serves, Sec. 4.1), in the predictor-evaluate-corrector form of Makino &
 * Aarseth (1992), on FP64 state:
 *   x_p = x + v dt + a dt^2/2 + j dt^3/6,  v_p = v + a dt + j dt^2/2,
 *   (a1, j1) = force and jerk at (x_p, v_p)   (nbody_force_jerk_f64 arithmetic),
 *   v' = v + (a + a1) dt/2 + (j - j1) dt^2/12,  x' = x + (v + v') dt/2 + (a - a1) dt^2/12,
 *   (a, j) <- (a1, j1).
 *   pos64, vel64  double [3][n], advanced nsteps steps in place
 *   acc, jerk     double [3][n]: a and j at the entry state (or computed first when
 *                 flags has NBODY_LF_INIT_ACC); on return those of the last evaluation,
 *                 which the next call continues from
 *   opts          precision, centre (as nbody_force_jerk_f64), ipl, jtile, nseg,
 *                 workspace (nbody_workspace_size_hermite bytes)
 * One force-jerk evaluation per step.  nbody_graph_create_hermite captures nsteps steps
 * (without the initial evaluation) into a graph that owns its scratch; replay it with
 * nbody_graph_launch and free it with nbody_graph_destroy. */
NBODY_API nbody_status nbody_hermite(int64_t n, double *pos64, double *vel64, const float *mass,
                                     float eps, double dt, int32_t nsteps, double *acc,
                                     double *jerk, int32_t flags, const nbody_opts *opts,
                                     void *stream);
NBODY_API nbody_status nbody_graph_create_hermite(int64_t n, double *pos64, double *vel64,
                                                  const float *mass, float eps, double dt,
                                                  int32_t nsteps, double *acc, double *jerk,
                                                  const nbody_opts *opts, void *stream,
                                                  nbody_graph **out);
NBODY_API size_t nbody_workspace_size_hermite(int64_t n, const nbody_opts *opts);

/* ------------------------------------------------------------------------------
 * Adjoint (vector-Jacobian product) of one force evaluation.  Given cotangents
 * g = dL/da and p = dL/dphi it returns, with d = x_j - x_k, s^2 = |d|^2 + eps^2,
 * w = m_k g_j - m_j g_k and q = m_k p_j + m_j p_k (sums over j != k):
 *     grad_pos_k  = sum_j [ w / s^3 - 3 (d . w) d / s^5 - q d / s^3 ]
 *     grad_mass_k = -sum_j [ (g_j . d) / s^3 + p_j / s ]
 * the derivative of eq. (1) and of the potential with respect to positions and masses.
 *   g_acc      double [3][n] (read)          g_pot   double [n] or NULL (= 0)
 *   grad_pos   double [3][n] (written)       grad_mass double [n] or NULL (skipped)
 * Pair arithmetic FP32 (positions as in nbody_force / nbody_force_f64), accumulation
 * per opts->precision, FP64 reduction.
 * ---------------------------------------------------------------------------- */
NBODY_API nbody_status nbody_force_vjp(int64_t n, const float *pos, const float *mass, float eps,
                                       const double *g_acc, const double *g_pot, double *grad_pos,
                                       double *grad_mass, const nbody_opts *opts, void *stream);
NBODY_API nbody_status nbody_force_vjp_f64(int64_t n, const double *pos64, const float *mass,
                                           float eps, const double *g_acc, const double *g_pot,
                                           double *grad_pos, double *grad_mass,
                                           const nbody_opts *opts, void *stream);
/* Bytes of scratch that nbody_force_vjp and nbody_force_vjp_f64 need (the adjoint's
 * own launch shape), and that nbody_leapfrog_adjoint needs (3n doubles more, for the
 * cotangent of the accelerations).  0 for n <= 0 or invalid options. */
NBODY_API size_t nbody_workspace_size_vjp(int64_t n, const nbody_opts *opts);
NBODY_API size_t nbody_workspace_size_adjoint(int64_t n, const nbody_opts *opts);

/* Reverse pass of nsteps KDK steps (nbody_leapfrog) from the checkpoints it stored.
 *   traj   double [nsteps+1][3][n]: x_0 .. x_nsteps (read)
 *   xbar   double [3][n]: on entry dL/dx_nsteps, on exit dL/dx_0
 *   vbar   double [3][n]: on entry dL/dv_nsteps, on exit dL/dv_0
 *   mbar   double [n] or NULL: dL/dm (through the dynamics) is ADDED to it
 * The cotangents of a(x_t) from the two kicks that use it are summed before one VJP
 * (nbody_force_vjp_f64 with the same options) per checkpoint.  nsteps = 0 leaves
 * xbar, vbar and mbar as they are (the rollout is the identity).  Scratch:
 * nbody_workspace_size_adjoint bytes. */
NBODY_API nbody_status nbody_leapfrog_adjoint(int64_t n, const double *traj, const float *mass,
                                              float eps, double dt, int32_t nsteps, double *xbar,
                                              double *vbar, double *mbar, const nbody_opts *opts,
                                              void *stream);

/* ------------------------------------------------------------------------------
 * Ragged batches: nsys independent systems stored back to back in one set of arrays;
 * system k owns the particles [offsets[k], offsets[k+1]) and interacts only with
 * itself (eq. (1) within each system), with its own softening eps[k].
 *
 * A plan is built once from the HOST array offsets (int64, nsys + 1 entries,
 * offsets[0] = 0, non-decreasing, total < 2^30; empty systems allowed).  It cuts every
 * system into work items (an i-tile against a j-range), sorts them by decreasing
 * cost, and owns the device tables, the partial-sum scratch and the ticket counter of
 * the persistent kernel that runs them - so every call with a plan allocates nothing
 * and can be captured in a graph.  Calls with the same plan must not overlap in time
 * (they share its scratch).  opts: precision, centre (NONE or SYSTEM), ipl, jtile;
 * self_pot must be 0 and workspace NULL.  The plan belongs to the current device.
 * ---------------------------------------------------------------------------- */
typedef struct nbody_plan nbody_plan;
NBODY_API nbody_status nbody_plan_create_batched(int32_t nsys, const int64_t *h_offsets,
                                                 const nbody_opts *opts, nbody_plan **out);
NBODY_API void nbody_plan_destroy(nbody_plan *plan);
/* info[0..8): nsys, total particles, work items, persistent blocks, pairs (sum N_k^2),
 * pairs including tile padding, ipl, jtile. */
NBODY_API nbody_status nbody_plan_info(const nbody_plan *plan, int64_t *info);

/* Forces and potentials of every system.  pos float [3][total], mass float [total],
 * eps float [nsys] (device), acc double [3][total], pot double [total] or NULL. */
NBODY_API nbody_status nbody_force_batched(const nbody_plan *plan, const float *pos,
                                           const float *mass, const float *eps, double *acc,
                                           double *pot, void *stream);
/* As nbody_force_batched with FP64 positions (converted per system relative to its
 * FP64 mean position when the plan's centre is NBODY_CENTRE_SYSTEM). */
NBODY_API nbody_status nbody_force_batched_f64(const nbody_plan *plan, const double *pos64,
                                               const float *mass, const float *eps, double *acc,
                                               double *pot, void *stream);
/* nsteps KDK leapfrog steps of every system at once (as nbody_leapfrog). */
NBODY_API nbody_status nbody_leapfrog_batched(const nbody_plan *plan, double *pos64,
                                              double *vel64, const float *mass, const float *eps,
                                              double dt, int32_t nsteps, double *acc, double *pot,
                                              int32_t flags, void *stream);
/* HIP graph of nsteps batched leapfrog steps (acc must hold a(pos64) when launched);
 * launched and destroyed with nbody_graph_launch / nbody_graph_destroy. */
NBODY_API nbody_status nbody_graph_create_leapfrog_batched(const nbody_plan *plan, double *pos64,
                                                           double *vel64, const float *mass,
                                                           const float *eps, double dt,
                                                           int32_t nsteps, double *acc,
                                                           double *pot, void *stream,
                                                           nbody_graph **out);

/* ------------------------------------------------------------------------------
 * Launch-shape table.  Shapes (i-particles per lane, j-tile, j-segments) are looked
 * up per kernel, precision mode and size bucket floor(log2 n) (batched: mean system
 * size); entries not set use built-in defaults; explicit opts fields override both.
 * The autotuner (tune.py) measures shapes and writes the JSON file these functions
 * read and write.  nseg = 0 lets the library choose the j-split from n.  The built-in
 * defaults use the split engine for the force below 2^13 particles.
 * ---------------------------------------------------------------------------- */
#define NBODY_KERNEL_FORCE 0
#define NBODY_KERNEL_VJP 1
#define NBODY_KERNEL_BATCHED 2
#define NBODY_KERNEL_JERK 3
NBODY_API nbody_status nbody_tune_set(int32_t kernel, int32_t precision, int64_t n, int32_t ipl,
                                      int32_t jtile, int32_t nseg, int32_t jlanes,
                                      int32_t symmetric);
/* shape[0..5) = ipl, jtile, nseg, jlanes, symmetric in effect for (kernel, precision,
 * n) (jlanes 1: grid engine; 8 to 64: split engine, only for NBODY_KERNEL_FORCE and
 * NBODY_KERNEL_VJP; symmetric 1: symmetric engine, only for NBODY_KERNEL_FORCE, with
 * jlanes 1).  shape must hold 5 values. */
NBODY_API nbody_status nbody_tune_get(int32_t kernel, int32_t precision, int64_t n,
                                      int32_t *shape);
NBODY_API nbody_status nbody_tune_load(const char *path);
NBODY_API nbody_status nbody_tune_save(const char *path);
NBODY_API void nbody_tune_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
