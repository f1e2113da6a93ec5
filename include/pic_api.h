/*
 * pic_api.h -- C ABI of the MI355X (gfx950) FDTD-Esirkepov PIC step with the
 * small-k_z correction stencils of Godfrey & Vay, "Suppressing the Numerical
 * Cherenkov Instability in FDTD PIC Codes" (arXiv:1401.0838).
 *
 * One step advances every bound simulation instance by dt:
 *   1. Yee update on the staggered mesh (Sec. 2 names the usual Yee mesh):
 *        B -= dt/2 curl E;  E += dt (curl B - J - J_bg);  B -= dt/2 curl E
 *   2. fields as seen by the particles (Sec. 2): Psi_E(S_z) on both transverse
 *      E components, Psi_B(S_z) on E_z and on every B component, with S_z the
 *      -(1/4)(1,-2,1) stencil along z whose symbol is s = sin^2(k_z dz/2);
 *      then the 3-point digital filter passes along every axis (Sec. 3, Eq. 6)
 *   3. per particle: Galerkin shape-factor gather (the scheme of Eq. 3: order l
 *      along axes where a component sits on integer nodes, l-1 where it sits
 *      half a cell off; Sec. 3), Boris push, move, Esirkepov deposit
 *      (the current-conserving scheme the paper's dispersion analysis assumes)
 *
 * Units: c = eps0 = mu0 = 1.  Positions are absolute (0 <= x < n*dx),
 * momenta are u = gamma*v per unit mass.  2D means the (x, z) plane with y
 * invariant and three velocity components; z is the beam axis.
 *
 * Memory: the caller owns one device arena (any allocator; the Python binding
 * uses a torch uint8 tensor) whose size pic_plan() reports.  The library keeps
 * every field, particle and tile array inside it and allocates no device
 * memory of its own.  A state is bound to one HIP stream and is not
 * thread-safe.  Every function returns PIC_OK (0) or a negative PIC_E* code
 * and never throws across the ABI.
 */
#ifndef PIC_API_H
#define PIC_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define PIC_OK            0
#define PIC_EINVAL       -1   /* bad argument, shape or order */
#define PIC_ECOURANT     -2   /* c dt >= 1 / sqrt(sum 1/d^2): Yee unstable */
#define PIC_EPSI         -3   /* Psi_B <= 0 somewhere on s in [0,1], Psi_E <= 0
                                 on [0,1) (at s = 1 it may vanish to rounding,
                                 as Eq. 5 does), or a singular interpolation
                                 system (Sec. 3 notes a breakdown window of the
                                 determination) */
#define PIC_ENOMEM       -4   /* arena smaller than pic_plan() asked for */
#define PIC_EHIP         -5   /* a HIP runtime call failed */
#define PIC_ENONFINITE   -6   /* pic_diag found a NaN or Inf */
#define PIC_EPARTICLE    -7   /* a particle moved a full cell or more in a step */
#define PIC_EUNSUPPORTED -8   /* valid but not built (e.g. the reverse sweep of a
                                 non-Galerkin gather) */
#define PIC_ESTATE       -9   /* call not valid in the current state */
#define PIC_ERANGE      -10   /* float mode: a current value left the checked range of
                                 the 32-bit fixed-point current planes (at least 2^9
                                 times the current of a beam moving at c through the
                                 densest cell of the initial load); the run's current
                                 is wrong */

/* ------------------------------------------------------------- enumerations */
/* gather (interpolation) schemes, with the multiplier each one's Psi fits */
#define PIC_GALERKIN 0        /* Eq. 3: order l, lowered by one along axes where
                                 the component sits half a cell off the nodes */
#define PIC_UNIFORM  1        /* Eq. 4: order l on every axis, from each
                                 component's own Yee location */
#define PIC_MOMENTUM 2        /* Eq. 5: seen fields averaged from the Yee mesh
                                 onto the integer nodes, then order l on every
                                 axis; PIC_FIELD_SEEN_E/B then read the node
                                 values, and every seen stencil is one cell
                                 wider (filter_npass <= 7) */

/* correction modes (Sec. 2) */
#define PIC_CORR_NONE  0      /* fields seen by the particles are only filtered */
#define PIC_CORR_SPLIT 1      /* Psi_E on the transverse E, Psi_B on E_z and B
                                 (the Sec. 2 approach, Psi_B acting as a filter) */
#define PIC_CORR_RATIO 2      /* the full Psi_E / Psi_B on the transverse E only,
                                 Psi_B inverted along z (Sec. 2's tri-diagonal
                                 route; a Sec. 3 variant); E_z and B are filtered
                                 only; needs nz <= 1024, Psi_B with real roots,
                                 forward runs only */

/* field solvers (Faraday's law; Ampere's law is always the Yee one) */
#define PIC_YEE 0             /* textbook Yee */
#define PIC_CK  1             /* Cole-Karkkainen with beta = 1/8 (named in Secs. 2-4):
                                 2D, square cells (dx == dz), c dt < dx, forward
                                 and reverse runs; every
                                 forward difference of E in Faraday's law is the
                                 (1/8, 3/4, 1/8) mean of that difference on its
                                 line and the two neighbouring lines across it */

#define PIC_FP64 0            /* fields, offsets, momenta and J in double */
#define PIC_FP32 1            /* float fields/offsets/momenta, int32 cell index;
                                 J summed per tile in fixed point — 64-bit in 2D
                                 (quantum 2^-28 of the largest single-particle
                                 contribution), 32-bit in 3D with a per-tile quantum
                                 that keeps every sum of the tile's particles below
                                 2^30 — and kept in HBM as 32-bit fixed point (quantum
                                 about 2^-21 of the current of a beam moving at c
                                 through the densest initial cell; each tile's sum is
                                 rounded to it once per step).  Integer sums: a run is
                                 bitwise reproducible for a given particle tiling */

#define PIC_IONS_CHARGE             0  /* immobile ions carry charge only */
#define PIC_IONS_CHARGE_AND_CURRENT 1  /* plus a fixed uniform current equal to
                                          minus the beam's initial mean current */

/* field selectors for pic_fields */
#define PIC_FIELD_E      0    /* E^n on the Yee mesh */
#define PIC_FIELD_B      1    /* B^n */
#define PIC_FIELD_J      2    /* J^{n+1/2} deposited by the last step */
#define PIC_FIELD_SEEN_E 3    /* E as seen by the particles in the last step */
#define PIC_FIELD_SEEN_B 4    /* B as seen by the particles in the last step */
#define PIC_FIELD_RHO    5    /* charge density of the current particles (comp 0) */

#define PIC_GET 0
#define PIC_SET 1

#define PIC_SCHED_BATCHED 0   /* every kernel launched once over all instances */
#define PIC_SCHED_PLAIN   1   /* each kernel launched once per instance */

/* ----------------------------------------------------------- configuration */
typedef struct pic_config {
    int    dims;              /* 2 (x, z) or 3 (x, y, z) */
    int    nx, ny, nz;        /* cells per axis, periodic; ny must be 1 in 2D */
    double dx, dy, dz;        /* cell sizes (dy ignored in 2D) */
    double cdt;               /* c * dt */
    int    shape_order;       /* charge shape order l: 1 or 3 */
    int    interp;            /* PIC_GALERKIN, PIC_UNIFORM or PIC_MOMENTUM; equal
                                 for all instances; the reverse sweep is built
                                 for PIC_GALERKIN and PIC_UNIFORM */
    int    precision;         /* PIC_FP64 or PIC_FP32; equal for all instances */
    int    correction;        /* PIC_CORR_NONE, PIC_CORR_SPLIT or PIC_CORR_RATIO; the
                                 ratio choice is equal for all instances */
    int    psi_deg;           /* polynomial degree of Psi_E and Psi_B, <= 8 */
    double psi_e[9];          /* Psi_E(s) = sum_j psi_e[j] s^j, psi_e[0] = 1 */
    double psi_b[9];          /* Psi_B(s) = sum_j psi_b[j] s^j, psi_b[0] = 1 */
    int    filter_npass;      /* 3-point passes per axis, <= 8 */
    double filter_w[8];       /* pass j is (w, 1-2w, w): 0.25 bilinear, -1 compensation */
    double q, m;              /* species charge and mass */
    double weight;            /* macro-particle weight (real particles per macro-particle
                                 per unit cell volume times cell volume) */
    int    ion_mode;          /* PIC_IONS_* */
    int    tile[3];           /* particle tile in cells along x, y, z (0 = default: 2D 16 x 16, or
                                 8 x 8 when the whole batch has fewer than 1024 default tiles;
                                 3D 8x4x4 linear, 8x2x4 cubic) */
    int    block;             /* threads per particle workgroup: 0 (default), 256 or 512 */
    int    trace_capacity;    /* steps of per-step field-energy trace kept on the device */
    int    adjoint_steps;     /* longest gradient run pic_adjoint_forward may do (0: none) */
    int    adjoint_ckpt;      /* checkpoint interval of gradient runs (steps, >= 1) */
    int    solver;            /* PIC_YEE or PIC_CK; equal for all instances */
} pic_config;

/* particles of one instance as host float64 arrays (structure of arrays) */
typedef struct pic_particles {
    int64_t       n;
    const double *pos[3];     /* absolute x, y, z positions; pos[1] ignored in 2D */
    const double *mom[3];     /* u_x, u_y, u_z */
} pic_particles;

typedef struct pic_diag_t {
    double  WE[3], WB[3];     /* 1/2 sum E_c^2 dV and 1/2 sum B_c^2 dV (E^n, B^n) */
    double  Wkin;             /* sum w m (gamma - 1) over particles (u^{n+1/2}) */
    double  gauss_l2;         /* ||(div E - rho) - (div E - rho)_initial||_2 on nodes */
    double  gauss_linf;       /* same, max norm; both at the particles' time level */
    double  charge;           /* sum rho dV */
    double  rho_max;          /* max |rho| (scale for the Gauss residual) */
    int64_t n_particles;
    int64_t step;             /* steps taken since pic_init */
    int     nonfinite;        /* 1 if any field or momentum is NaN / Inf */
    int     particle_error;   /* 1 if a particle moved a full cell or more */
    int     resorts;          /* tile re-sorts done since pic_init */
    int     slow_tiles;       /* tile visits that overflowed the LDS window */
    int     current_range;    /* 1 if a float-mode current value left its checked range */
} pic_diag_t;

/* per-kernel average durations measured with HIP events (milliseconds) */
typedef struct pic_timing_t {
    double yee_ms, seen_ms, particle_ms, resort_ms, step_ms;
    int    steps;
} pic_timing_t;

struct pic_state;
typedef struct pic_state pic_state;

/* Correction-stencil coefficients (Sec. 2): the power-series coefficients of
 * Psi_E and Psi_B in s = sin^2(k_z dz/2), from rational interpolation of the
 * multiplier of Eq. 3 (PIC_GALERKIN), Eq. 4 (PIC_UNIFORM) or Eq. 5
 * (PIC_MOMENTUM) at 2*deg+1 nodes spaced uniformly on s in [0, 1]
 * (9 nodes, quartics, for deg = 4), with psi_b[0] = 1.  alpha = c dt / dz.
 * Solved in 113-bit binary floating point and rounded to double.  Returns
 * PIC_EPSI if the system is singular (except where the multiplier is
 * identically 1, which gives Psi_E = Psi_B = 1), if Psi_B <= 0 somewhere on
 * s in [0, 1], or if Psi_E <= 0 on [0, 1).  At s = 1 the Eq. 5 multiplier is
 * exactly 0, so Psi_E(1) is accepted down to -1e-12 sum |psi_e[i]|.  Writes
 * deg+1 doubles to each output. */
int pic_psi_coeffs(int interp, double alpha, int deg, double *psi_e, double *psi_b);

/* Size in bytes of the device arena for n_inst instances with the given
 * particle counts. */
int pic_plan(const pic_config *cfgs, int n_inst, const int64_t *n_particles, size_t *arena_bytes);

/* Set up the problem Sec. 3 simulates: a uniform relativistic beam drifting
 * along z through a periodic box on the Yee mesh of Sec. 2, with the
 * correction polynomials Psi_E / Psi_B of Sec. 2 (psi_e, psi_b; see
 * pic_psi_coeffs), the digital filter of Sec. 3 / Eq. 6 (filter_w; Sec. 4's
 * variant with one pass of each kind is the same list with two entries), the
 * gather scheme whose multiplier Eqs. 3-5 give, and the time step
 * alpha = c dt / dz that Secs. 3-4 scan.
 * Validate the configurations, lay them out in the arena, upload the
 * particles (host float64 -> device; converted to cell index + in-cell
 * offset), sort them by tile and record the initial charge density.
 * d_arena: device pointer of arena_bytes bytes (256-byte aligned), owned by
 * the caller and kept alive until pic_destroy.  hip_stream: hipStream_t or
 * NULL for the default stream.  Blocks until the upload is complete. */
int pic_init(const pic_config *cfgs, int n_inst, const pic_particles *parts,
             void *d_arena, size_t arena_bytes, void *hip_stream, pic_state **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): pic_init with the
 * arena taken from a static device array of PIC_STATIC_ARENA_BYTES that the
 * library holds on every device it runs on until the process ends (64 MiB: one
 * 2D FP32 instance of 256 x 256 cells at 8 particles per cell needs 41 MiB).
 * Arguments as for pic_init less the arena; hip_stream must be a stream of the
 * current device (NULL is rejected: no stream is created).  Allocates no device
 * memory.  The array holds one state per device: while a state made by this
 * call on a device is alive, a further call there returns PIC_ESTATE (calls
 * that overlapped on one device would otherwise overwrite each other's state);
 * pic_destroy releases the array.  Each call clears what the scheme needs at
 * zero, as pic_init does.  PIC_ENOMEM when pic_plan asks for more than
 * PIC_STATIC_ARENA_BYTES. */
#define PIC_STATIC_ARENA_BYTES (64u << 20)
int pic_init_static(const pic_config *cfgs, int n_inst, const pic_particles *parts, void *hip_stream,
                    pic_state **out);

/* Advance every instance by nsteps steps of the explicit scheme Sec. 2
 * analyses: the Yee field update, then the fields as seen by the particles
 * (Psi_E(S_z) on the transverse E and Psi_B(S_z) on the rest, Sec. 2,
 * followed by the filter passes of Sec. 3 / Eq. 6), then per particle the
 * gather of those fields, the Boris push, the move and the current-conserving
 * deposit.  Asynchronous on the bound stream. */
int pic_step(pic_state *st, int nsteps);

/* Capture (without running) the HIP graphs that a following
 * pic_step(st, nsteps) from the current state replays, so that call pays no
 * capture (for timed regions and serving loops).  With graph replay a call
 * launches at most three kinds of graph: the steps up to the next re-sort
 * check, whole re-sort periods, and the rest; graphs are cached until the
 * schedule or an option changes.  Synchronous; a no-op for eager stepping. */
int pic_prepare(pic_state *st, int nsteps);

/* Choose the launch schedule (PIC_SCHED_*) and whether steps are replayed
 * from a captured HIP graph (use_graph = 1) or launched eagerly. */
int pic_set_schedule(pic_state *st, int sched, int use_graph);

/* Tuning knobs (used by the autotuner); every one keeps results unchanged:
 *   "yee_tile_z"     rows of the 2D Yee tile: 4, 8 or 16 (16 is float only);
 *                    default 8, or 16 for FP32 batches of more than 4 * 512^2 cells
 *   "seen_tile_z"    rows of the 2D seen-field tile: 8, 16, 32 or 64 (32 and 64
 *                    are float only), or 128: float strips 128 columns wide and
 *                    128 rows tall streamed in 32-row chunks (with the usual
 *                    stencil widths, else 32);
 *                    default 16, or 128 (32 where the widths differ) for FP32
 *                    batches of more than 4 * 512^2 cells
 *   "resort_every"   steps between tile re-sort checks (and per captured graph);
 *                    default 16
 *   "particle_block" threads per particle workgroup: 256 or 512
 *   "particle_waves4" 1: 2D linear float particle kernel built for four waves
 *                    per SIMD (register cap 128)
 *   "particle_prefetch" 1: 2D linear float particle kernel loads the next
 *                    particle's state while pushing the current one
 *   "particle_defer" 2D: 0 steps a tile whose particles outgrew its LDS window
 *                    inside the particle kernel; 1 leaves such tiles to a second
 *                    launch (fewer registers in the first, more waves per SIMD);
 *                    -1 (default) picks 1 when there are more than four tiles per
 *                    compute unit.  3D always uses the second launch.
 * Returns PIC_EINVAL for an unknown name or value.  Drops captured graphs. */
int pic_set_option(pic_state *st, const char *name, int value);
int pic_get_option(pic_state *st, const char *name, int *value);

/* Grid fields of the scheme: E and B on the Yee mesh (Sec. 2), the fields as
 * seen by the particles after the correction and filter (Sec. 2: the
 * multipliers act on what the particles see, not on the grid fields), J and
 * the charge density.
 * Copy one component of a grid quantity (PIC_FIELD_*) of instance inst to
 * (GET) or from (SET) a host float64 array of n = nx*ny*nz values laid out
 * [z][y][x], x fastest, half-integer locations stored at the lower index.
 * SET is allowed for E and B only.  Synchronises the stream. */
int pic_fields(pic_state *st, int inst, int which, int comp, double *host, size_t n, int dir);

/* Copy the particles of instance inst to host float64 arrays in the order
 * they were given to pic_init (absolute positions wrapped into the box).
 * pos[1] may be NULL in 2D.  Synchronises the stream. */
int pic_get_particles(pic_state *st, int inst, double *pos[3], double *mom[3], int64_t n);

/* Diagnostics of instance inst (float64 reductions on the device): the field
 * energies whose transverse part gives the growth rates of Sec. 3 and whose
 * total Sec. 4 tracks, the beam's kinetic energy, and the Gauss-law residual
 * that the current-conserving deposit keeps at rounding level.
 * Synchronises the stream.  Returns PIC_ENONFINITE, PIC_EPARTICLE or PIC_ERANGE
 * when the corresponding flag is set (out is filled in either case). */
int pic_diag(pic_state *st, int inst, pic_diag_t *out);

/* Per-step transverse and total field energies recorded since pic_init when
 * trace_capacity > 0: host_out receives count rows of 6 doubles
 * (WE_x, WE_y, WE_z, WB_x, WB_y, WB_z) for the last min(steps, capacity) steps
 * in step order; *count is set to the number of rows written. */
int pic_read_trace(pic_state *st, int inst, double *host_out, int max_rows, int *count);

/* Run nsteps steps with HIP events around every kernel of the step and
 * report average durations.  Synchronises the stream. */
int pic_profile(pic_state *st, int nsteps, pic_timing_t *out);

/* Reverse mode: gradient of the late-time transverse field energy
 *   W = 1/2 sum (E_x^2 + E_y^2 + B_x^2 + B_y^2) dV   after nsteps steps
 * with respect to the Psi_E coefficients psi_e[0..psi_deg] of every instance
 * (Sec. 2 defines Psi_E; tuning its coefficients is the use).
 *
 * pic_adjoint_forward runs nsteps steps from the current state, saving a
 * checkpoint every adjoint_ckpt steps, and writes W of instance i to loss[i].
 * Tile re-sorting is suspended until the matching backward call.  Requires
 * correction = 1 and nsteps <= adjoint_steps for every instance.
 *
 * pic_adjoint_backward then runs the reverse sweep: every segment is
 * recomputed from its checkpoint while its per-step tape is recorded, and its
 * steps are reversed with hand-written adjoint kernels (exact transposes of
 * the Yee update, the correction and filter stencils, the gather, the Boris
 * push, the move and the Esirkepov deposit).  In 2D a segment is recomputed
 * on the bound stream while the one after it is reversed on a second stream
 * (default priority, created by the first call and kept until pic_destroy);
 * the arena holds two segments of tape for that.  grad[i*9 + j] receives
 * dW/dpsi_e[j] of instance i (zero for j > psi_deg).  On return the state is
 * again the forward state after the nsteps steps.  Both calls synchronise. */
int pic_adjoint_forward(pic_state *st, int nsteps, double *loss);
int pic_adjoint_backward(pic_state *st, double *grad);

/* Number of instances, and the total particle count over all instances. */
int pic_info(pic_state *st, int *n_inst, int64_t *n_particles, int64_t *n_cells);

void pic_destroy(pic_state *st);

/* Static description of a status code. */
const char *pic_strerror(int code);

/* Text of the most recent error on this thread (HIP error names included). */
const char *pic_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PIC_API_H */
