/*
 * mclbm.h -- C ABI of libmclbm, the MI355X (gfx950) implementation of the time
 * step of the consistent multicomponent lattice Boltzmann model of Sawant,
 * Dorschner and Karlin (arXiv 2004.11286): M species population sets relaxing
 * under the Stefan--Maxwell kinetic model (Sec. 2), a compressible mixture
 * momentum lattice and an energy lattice (Sec. 3), all on D3Q27, strongly
 * coupled (Sec. 3.5.2) or weakly coupled (Sec. 3.5.1), fused stream-and-collide
 * over every node; x ends periodic, walled or open; constant or
 * temperature-dependent specific heats and transport coefficients.
 *
 * Conventions for every call:
 *   - Return value: MCLBM_OK (0) on success, a negative MCLBM_E* code on error;
 *     mclbm_last_error() then describes the failure. No exception crosses the ABI.
 *   - Units: lattice units, dt = dx = 1, universal gas constant R_U = 1 (a species
 *     of molar mass m_a has gas constant 1/m_a), T_0 = 0 (Sec. 4.1); specific
 *     heats constant unless mclbm_params.cv_coef is given. Physical data are
 *     converted by acoustic scaling in the Python package (units.py).
 *   - Field layout: structure of arrays, x fastest: node n = x + nx (y + ny z).
 *     A field with C components is C consecutive planes of nx*ny*nz doubles.
 *   - Ownership: the caller owns every buffer it passes, including the device
 *     workspace; the library never frees them. The context is owned by the
 *     library (mclbm_destroy).
 *   - Streams: every call is ordered on the HIP stream given at creation; calls
 *     that return data to the host synchronise that stream. Calls on one context
 *     are not thread safe.
 *   - Under strong coupling (the default) one species is slaved to the mixture
 *     (Sec. 3.5.2): its density and momentum are the deficits of the mixture's.
 *     mclbm_params.slaved names it (default species M); choose one that carries
 *     most of the mass everywhere. Under weak coupling (mclbm_params.weak) every
 *     species has its own lattice.
 *   - Batches: a context holds one or more independent lattices ("tubes", the
 *     Loschmidt-tube setting of Sec. 4.2 repeated with different mixtures). All
 *     tubes of a context share M, wall_x, precision, the coupling and which
 *     optional data are given; sizes, species data and inlets differ per tube. Every per-node array of the calls below is the
 *     concatenation over the tubes, in creation order, of that tube's own array
 *     in the single-tube layout: a field with C components holds, for tube t,
 *     C * n_t values at offset C * (n_0 + ... + n_{t-1}). A context made with
 *     mclbm_create is a batch of one tube.
 */
#ifndef MCLBM_H
#define MCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes */
#define MCLBM_OK 0
#define MCLBM_EARG (-1)        /* invalid argument or size                         */
#define MCLBM_ESTATE (-2)      /* infeasible state (T <= 0, R_a T + u^2 >= 1, ...) */
#define MCLBM_EDEVICE (-3)     /* HIP runtime error                                */
#define MCLBM_ENAN (-4)        /* non-finite value or negative slaved density      */
#define MCLBM_EUNSUPPORTED (-6)/* configuration not compiled into this library     */

/* Storage and arithmetic precision of the populations (mclbm_params.precision). */
#define MCLBM_FP64 0      /* FP64 storage, FP64 collision                                   */
#define MCLBM_FP32 1      /* FP32 storage, FP64 collision (same FMA rate as non-packed FP32) */
#define MCLBM_FP32_FP32 2 /* FP32 storage, FP32 collision                                   */
#define MCLBM_FP16 3      /* FP16 storage of scaled deviations, FP32 collision               */
#define MCLBM_BF16 4      /* BF16 storage of scaled deviations, FP32 collision               */
#define MCLBM_I16 5       /* 16-bit fixed-point storage of deviations, FP32 collision (below) */
/* MCLBM_I16 stores every population of lattice l, direction i as a 16-bit
 * integer v with f = f_ref + v h / 32767, where f_ref and the half-width h are
 * shared by the directions of a class (equal |c_x|, |c_y|, |c_z|), per lattice
 * and tube; stores round stochastically. mclbm_init_fields measures the range
 * each class takes in the initial state and in the 4 steps after it (run with
 * wide tables and discarded: the transient of a sharp initial state), and fits
 * f_ref to its middle and h to twice its half-spread, at least |f_ref|.
 * mclbm_step reads a device flag per tube after steps 1, 2, 4 and every multiple
 * of 8 (the step count alone sets these points, so the trajectory does not
 * depend on how steps are split into calls or launched, and a tube of a batch
 * evolves as it would alone; checkpoints keep the flags): when a value of a tube
 * passed 3/4 of its range, that tube's tables are fitted to its current state
 * again and its state is re-encoded (mclbm_range_refits counts this); when a
 * value was clamped at the end of its range or was not finite, mclbm_step
 * returns MCLBM_ESTATE and the state is lost. Strong and weak coupling, constant
 * properties, periodic or walled x ends. The paper fixes no storage precision;
 * this is a storage format of this library. */

/* Kernel identifiers for mclbm_kernel_stats. */
#define MCLBM_K_MOMENTS 0  /* moments of every lattice -> node record {Phi, omega, C_p} */
#define MCLBM_K_GFIELD 1   /* G_a = (1/omega - 1/2) d_a Phi_a (inner derivative of eq Xalpha) */
#define MCLBM_K_COLLIDE 2  /* collisions of all lattices + streaming                      */

typedef struct mclbm_ctx mclbm_ctx;

/* Problem description. Arrays are read during mclbm_create only. */
typedef struct {
  int32_t M;           /* species count (the kernels are compiled for 2, 3 and 4)      */
  int32_t nx, ny, nz;  /* lattice size; nx*ny*nz < 2^31                               */
  int32_t wall_x;      /* 0: periodic in x; 1: half-way bounce-back walls at both x ends
                          (Sec. 4.2); 2: open x ends, an equilibrium inlet at x = 0 (the
                          populations entering node 0 are the local equilibrium of the
                          fields `inlet`) and a zero-gradient outlet at x = nx - 1 (the
                          populations entering it are the boundary node's post-collision
                          values), both as in the opposed jets of Sec. 4.3; open ends
                          are compiled for MCLBM_FP64 and MCLBM_FP32 (else
                          MCLBM_EUNSUPPORTED), with either coupling and either kind of
                          properties. 3: the opposed jets of Sec. 4.3: on both x faces
                          the rows nozzle_y0 <= y < nozzle_y1 are equilibrium inlets
                          (`inlet` at x = 0, `inlet_right` at x = nx - 1) and the other
                          rows free-slip walls (specular reflection); needs wall_y = 2,
                          strong coupling, constant properties, MCLBM_FP64 or MCLBM_FP32
                          (else MCLBM_EUNSUPPORTED). z is always periodic; y is
                          periodic unless wall_y */
  int32_t precision;   /* MCLBM_FP64 .. MCLBM_I16                                     */
  int32_t weak;        /* 0: strong coupling (Sec. 3.5.2): species M is slaved to the
                          momentum lattice (eqs rhoMATCH, uMATCH) and not stored.
                          1: weak coupling (Sec. 3.5.1): all M species lattices are
                          stored and evolved; the species keep their own density and
                          velocity (eqs rhoSPEC, uSPEC) and Dalton pressure, and take
                          T from the energy lattice. MCLBM_FP64, MCLBM_FP32,
                          MCLBM_FP16 and MCLBM_I16 (else MCLBM_EUNSUPPORTED); all
                          tubes of a batch agree                                    */
  int32_t wall_y;      /* 0: periodic in y; 1: free-slip walls at both y ends (half-way,
                          specular reflection), with periodic or walled x ends, either
                          coupling and either kind of properties; MCLBM_FP64 and
                          MCLBM_FP32 (else MCLBM_EUNSUPPORTED). 2: zero-gradient outlets
                          at both y ends (what enters comes from a ghost row holding
                          the boundary row's post-collision state: the outlets of the
                          opposed jets, Sec. 4.3), only with wall_x = 3. All tubes of
                          a batch agree                                              */
  const double *molar_mass;  /* [M] molar masses m_a > 0                              */
  const double *cv;          /* [M] mass-based specific heats C_{a,v} > 0             */
  const double *D;           /* [M*M] symmetric binary diffusivities D_ab > 0, row major,
                                diagonal included (the sums of eqs tau and fStar run over
                                b = a)                                                 */
  const double *mu;          /* [M] species dynamic viscosities (Wilke mixing, Sec. 3.3) */
  const double *lambda;      /* [M] species thermal conductivities (Mathur mixing)    */
  const double *cv_coef;     /* NULL: constant specific heats cv (eq temperature2). Else
                                [M][4]: C_{a,v}(T) = sum_k c_ak T^k with c_a0 > 0 and
                                c_ak >= 0 (k >= 1), cv unused; U_a = int_0^T C_{a,v},
                                H_a = U_a + R_a T (eqs specUa, specHa) and T from
                                eq temperature by Newton's method (Sec. 3.1), with Y_a
                                the species subsystem's under weak coupling. MCLBM_FP64
                                or MCLBM_FP32 only (else MCLBM_EUNSUPPORTED); all tubes
                                of a batch agree on NULL                                */
  const double *inlet;       /* wall_x = 2: [M + 5] inlet fields X_1..X_M (sum 1), p, T,
                                u_x, u_y, u_z (each tube its own); else ignored         */
  const double *transport_exp; /* NULL: constant mu, lambda, D. Else [2M + 2]: s_mu (M),
                                s_lam (M), s_D, T_ref > 0, giving mu_a (T/T_ref)^s_mu,a,
                                lambda_a (T/T_ref)^s_lam,a, D_ab (T/T_ref)^s_D at the
                                local T (the given mu, lambda, D are the values at
                                T_ref); Wilke's phi from the viscosities at T. Same
                                support and batch rule as cv_coef                      */
  const double *inlet_right; /* wall_x = 3: [M + 5] fields of the jet entering at x = nx - 1
                                (X_1..X_M, p, T, u_x, u_y, u_z); else ignored           */
  int32_t nozzle_y0, nozzle_y1; /* wall_x = 3: the nozzle rows, 1 <= nozzle_y0 < nozzle_y1
                                <= ny - 1; else ignored                                 */
  int32_t slaved;      /* strong coupling: the species whose density and momentum
                          follow from the mixture's (eqs rhoMATCH, uMATCH; the paper
                          slaves the one carrying most of the mass), 1-based; 0 means
                          species M. The library keeps it last internally; every array
                          and field crossing this interface stays in the caller's
                          species order. Weak coupling: 0 (or M). All tubes of a batch
                          agree; mclbm_nn_advance takes only 0 (or M)             */
} mclbm_params;

/* Device workspace bytes a context with these parameters needs (0 on bad input). */
size_t mclbm_workspace_bytes(const mclbm_params *p);

/* Workspace bytes of a batch of ntubes independent tubes (0 on bad input). */
size_t mclbm_batch_workspace_bytes(const mclbm_params *tubes, int32_t ntubes);

/* Create a context on the current HIP device. dev_workspace: device memory of at
 * least mclbm_workspace_bytes(p) bytes, 256-byte aligned, borrowed until
 * mclbm_destroy. hip_stream: a hipStream_t (NULL = the null stream). */
int mclbm_create(const mclbm_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
                 mclbm_ctx **out);

/* Create a context over ntubes independent tubes (tubes[t] describes tube t;
 * M, wall_x and precision must agree). Workspace and stream as in mclbm_create.
 * Each step advances every tube; a tube's results are bit for bit those of a
 * context of that tube alone. */
int mclbm_batch_create(const mclbm_params *tubes, int32_t ntubes, void *dev_workspace, size_t bytes,
                       void *hip_stream, mclbm_ctx **out);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same context as
 * mclbm_create, whose workspace is instead an array of
 * MCLBM_STATIC_WORKSPACE_BYTES bytes inside the library, one per device, that
 * the device keeps until the process ends. No device memory is allocated (no
 * hipMalloc, no allocating library routine). Every call of the context works as
 * with mclbm_create. Limits: MCLBM_EARG (with a message naming the sizes) when
 * mclbm_workspace_bytes(p) exceeds the array; one context per device at a time
 * (MCLBM_EARG while another holds it; mclbm_destroy releases it). The array
 * keeps the last context's contents; a new context initialises whatever it
 * reads (mclbm_init_fields or mclbm_load), as with any workspace. The calls of
 * a static context race with those of any other context on the same device
 * only through this array, which no other context can hold; calls on one
 * context are not thread safe (as for every context). */
#define MCLBM_STATIC_WORKSPACE_BYTES (64u << 20)
int mclbm_create_static(const mclbm_params *p, void *hip_stream, mclbm_ctx **out);

void mclbm_destroy(mclbm_ctx *c);

/* Number of tubes, and total number of nodes over all tubes. */
int32_t mclbm_tube_count(const mclbm_ctx *c);
int64_t mclbm_node_count(const mclbm_ctx *c);

/* Message of the last error on this context; with c == NULL, of the last failed
 * mclbm_create or mclbm_workspace_bytes on this thread. */
const char *mclbm_last_error(const mclbm_ctx *c);

/* Set every lattice to the local equilibrium of the given fields (the paper is
 * silent on initial populations; the species k-populations equal the equilibria
 * there, Sec. 2.5.2 eq fixed). X [M][n] mole fractions (each node sums to 1),
 * p [n] pressure, T [n] temperature, u [3][n] velocity. on_device = 1: the four
 * pointers are device memory; 0: host memory. Resets the step counter. */
int mclbm_init_fields(mclbm_ctx *c, const double *X, const double *p, const double *T,
                      const double *u, int on_device);

/* Advance nsteps time steps, asynchronously on the context's stream. One step is
 * the species lattice Boltzmann equation of Sec. 2.5.3 (eqs SMlbm, fstar1,
 * transform12, with the moments of eqs densitya, momSPEC), the two-population
 * mixture equations of Sec. 3.2 (eq g with eqs gstareq1mom, interdiffusion,
 * corrFourier) realised on D3Q27 as in Sec. 3.4 (eqs gieq, gistar; the momentum
 * lattice with the correction of Sec. 3.4.2, eqs fwithcorrection, Xalpha, Ai),
 * coupled as in Sec. 3.5 (strong: eqs rhoMATCH, uMATCH), then streaming with the
 * boundary rules of mclbm_params. Every non-local term (eqs Xalpha, corrFourier)
 * uses the moments of the same time level. MCLBM_EARG before the first
 * initialisation or for nsteps < 0; MCLBM_EDEVICE if a launch fails. With
 * MCLBM_I16 storage it synchronises at each range check to read the range flags
 * (see MCLBM_I16) and returns MCLBM_ESTATE if a value left its range. */
int mclbm_step(mclbm_ctx *c, int64_t nsteps);

/* MCLBM_I16 storage: how many times mclbm_step fitted the tables to the state and
 * re-encoded it since the last mclbm_init_fields or mclbm_load (0 for other
 * storage); -1 for a NULL context. */
int64_t mclbm_range_refits(const mclbm_ctx *c);

/* Macroscopic fields of the current state (Secs. 2.1, 2.5.3, 3.2): X [M][n],
 * rho [n], u [3][n], p [n], T [n] as doubles; any pointer may be NULL. on_device
 * as in mclbm_init_fields. Synchronises the stream. */
int mclbm_read_moments(mclbm_ctx *c, double *X, double *rho, double *u, double *p, double *T,
                       int on_device);

/* The conserved fields of the step (eq DOF: the M species densities, or under
 * strong coupling M - 1 of them plus the mixture density, the mixture momentum
 * and the total energy of eq g0momTotalEnergy), summed over every node of each tube.
 * Domain sums in FP64 per tube, out [ntubes][M+5]: rho_1 .. rho_M (rho_M slaved
 * under strong coupling, from its own lattice under weak),
 * rho, rho u_x, rho u_y, rho u_z, rho E. Returns MCLBM_ENAN if any node holds a
 * non-finite value or a negative slaved density. Synchronises the stream. */
int mclbm_conservation(mclbm_ctx *c, double *out);

/* The fields a trajectory keeps, in FP32: out [M+5][n] per tube (X_1 .. X_M, T,
 * u_x, u_y, u_z, p), concatenated over tubes. on_device as in mclbm_init_fields.
 * Synchronises the stream. */
int mclbm_read_fields_f32(mclbm_ctx *c, float *out, int on_device);

/* Number of time steps since the last mclbm_init_fields or mclbm_load. */
int64_t mclbm_step_count(const mclbm_ctx *c);

/* Checkpoint: the population state, the reference tables and the step count,
 * copied to / from a host buffer of mclbm_state_bytes(c) bytes. Restoring into a
 * context created with the same parameters (M, boundaries, precision, coupling,
 * slaved species, property kinds and tube sizes are checked) resumes bit for bit. */
size_t mclbm_state_bytes(const mclbm_ctx *c);
int mclbm_save(mclbm_ctx *c, void *host_buf, size_t bytes);
int mclbm_load(mclbm_ctx *c, const void *host_buf, size_t bytes);

/* Per-kernel timing with HIP events recorded on the context's stream around each
 * launch of mclbm_step while enabled. mclbm_kernel_stats synchronises, returns the
 * summed milliseconds and launch count of kernel k (MCLBM_K_*) since timing was
 * enabled, and its name. */
int mclbm_set_timing(mclbm_ctx *c, int enable);
int mclbm_kernel_stats(mclbm_ctx *c, int32_t kernel, double *total_ms, int64_t *launches,
                       const char **name);

/* How mclbm_step launches its kernels. Every choice computes the same step. Within
 * one path (two-read or three-pass) the results are bit for bit the same (over
 * every block shape, tube order, swizzle and graph choice), except
 * split, whose two kernels are compiled separately and may fuse a multiply-add
 * differently: its results agree to rounding (and, with 16-bit storage, to the
 * stochastic rounding that such a last-bit difference can flip). The two paths
 * agree to the rounding of the stored state (the three-pass path carries the
 * node state through a record of the storage's record precision). Only the time
 * differs.
 *
 * The two-read step (three_pass = 0, where compiled: constant specific heats and
 * transport) launches per step: the moments of every lattice, which also collide
 * and stream the species lattices, whose collisions use only the node's own
 * moments (eqs SMlbm, fstar1, transform12); the stencil field G; the collision
 * and streaming of the momentum and energy lattices, whose non-local terms (eqs
 * Xalpha, corrFourier) need the neighbours' moments of the same time level. The
 * species populations are read once per step, f and g twice. The three-pass step
 * (three_pass = 1) reads every lattice twice: moments, stencil field, collision
 * of every lattice. */
typedef struct {
  int32_t variant;      /* occupancy variant of the moments kernel, and of the fused
                           collide kernel (split = 0), 0 or 1                           */
  int32_t swizzle;      /* 1: each XCD takes a contiguous run of blocks                  */
  int32_t order;        /* 0: tubes in the given order; 1: longest tube first            */
  int32_t graph_steps;  /* 0: launch each kernel of each step; K > 0 (even): replay a
                           HIP graph of K captured steps (not while timing is enabled)   */
  int32_t sequential;   /* 1: launch every tube on its own (the unbatched reference)     */
  int32_t split;        /* three-pass step only: 1: collide the species lattices, then
                           the momentum and energy lattices, in two launches with fewer
                           registers each (one occupancy form)                          */
  int32_t three_pass;   /* 1: the three-pass step; 0: the two-read step where compiled
                           (constant properties), else the three-pass step             */
  int32_t shape;        /* block shape of the step kernels' 256-thread blocks: 0 the
                           linear numbering (256 consecutive nodes, rows wrapping); tiles
                           of x * y * z nodes: 1 64x4x1, 2 32x8x1, 3 16x16x1, 4 64x2x2,
                           5 32x4x2 (threads beyond a tube's grid idle). Results are
                           bit for bit the same for every shape                          */
} mclbm_launch;

/* A new context starts with every field 0 (the two-read step where compiled),
 * except with temperature-dependent properties (the three-pass step), which starts
 * with split = 1, and under weak coupling also variant = 1 (the faster choices
 * there). */
int mclbm_get_launch(const mclbm_ctx *c, mclbm_launch *out);
int mclbm_set_launch(mclbm_ctx *c, const mclbm_launch *in);

/* Time the launch choices over trial_steps steps each on the current state and
 * keep the fastest: first every path (the two-read step with variant 0 or 1 where
 * compiled; the three-pass step with (variant, split) in {0,1}^2), each with
 * swizzle and HIP graph replay on or off, and for batches both tube orders, in
 * the linear block numbering; then the fastest of those with each tiled block
 * shape. Writes a text table of the candidates (milliseconds per step; columns
 * three_pass variant split swizzle order graph_steps shape) to report (may be
 * NULL), ending with the chosen line. The trial steps are ordinary steps: the
 * state and the step count advance by about (number of candidates) * 2
 * trial_steps. Synchronises the stream. */
int mclbm_autotune(mclbm_ctx *c, int32_t trial_steps, char *report, size_t report_len);

/* Moles of every species in each x half of every tube, FP64 (the diagnostic of
 * the Loschmidt tube, Sec. 4.2: half-tube mean mole fractions are the ratios of
 * these): out[t][h][a] = sum over the nodes of tube t with x < nx / 2 (h = 0) or
 * x >= nx / 2 (h = 1) of rho_a / m_a (R_U = 1, the slaved species' density from
 * the deficit of eq rhoMATCH). out: host [ntubes][2][M]. Synchronises the stream.
 * MCLBM_EARG before the first initialisation. */
int mclbm_half_tube_moles(mclbm_ctx *c, double *out);

/* Streaming copy of `bytes` bytes (a multiple of 16; both pointers 16-byte
 * aligned device memory, not overlapping) from src to dst, ordered on hip_stream
 * (NULL: the default stream): 16-byte nontemporal loads and stores, the access
 * kind of the population streams. It touches no lattice state; timing it gives the
 * read + write rate the memory sustains, the practical ceiling beside the peak
 * bandwidth. MCLBM_EARG for a bad size or alignment, MCLBM_EDEVICE if the launch
 * fails. */
int mclbm_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
