// Internal layout shared by the HIP kernels and the host orchestration.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PIC_MAX_HZ 16           // half-width of the combined z stencil (Psi degree + passes)
#define PIC_MAX_HX 8            // half-width of the x / y filter stencils
#define PIC_FIELD_CHUNK 256     // cells per field work item
#define PIC_SEEN_XSEG 8         // 64-cell row segments per wave of the 3D x-direction seen pass
#define PIC_GRAD_COPIES 64      // copies of the gradient sums (power of two)
#define PIC_PART_CHUNK 256      // particles per particle-chunk work item
#define PIC_SEEN_TX 64          // 2D seen-field tile (x)
#define PIC_SEEN_SW 128         // 2D streamed seen pass: strip width (x)
#define PIC_TILE_SLACK 4        // cells a tile's particle bounding box may grow before a re-sort
#define PIC_COL_RUN 16          // cells per thread along the axis of a 3D column stencil pass

// device flag slots (per instance)
// FLAG_JRANGE: a current sum left the 32-bit fixed-point range of the HBM planes (float mode)
enum { FLAG_RESORT = 0, FLAG_PERR = 1, FLAG_SLOW = 2, FLAG_NRESORT = 3, FLAG_JRANGE = 4, FLAG_COUNT = 8 };

// per-instance diagnostic accumulator slots (doubles)
enum {
    DG_WE = 0,      // 3
    DG_WB = 3,      // 3
    DG_WKIN = 6,
    DG_G2 = 7,      // sum of squared Gauss residual
    DG_GMAX = 8,    // max |residual| (bit pattern of a non-negative double)
    DG_CHARGE = 9,
    DG_RHOMAX = 10, // max |rho| (bit pattern)
    DG_NONFIN = 11, // > 0 if a non-finite value was seen
    DG_COUNT = 16
};

// Everything a kernel needs to know about one simulation instance.
struct InstDesc {
    int n[3];              // cells along x, y, z (n[1] = 1 in 2D)
    int ncell;
    int tile[3];           // particle tile size in cells
    int nt[3];             // tiles per axis
    int ntiles;
    int trace_cap;
    long long np;          // particles
    double d[3];           // cell sizes
    double dt;
    double dtd[3];         // dt / d_a
    double qdt2m;          // q dt / (2 m)
    double w, m;           // weight, mass
    double dV;
    double jbg[3];         // uniform background current
    double jq;             // fixed-point quantum of the LDS current sums (float mode): J = int64 * jq
    double jqg;            // quantum of the HBM current planes (float mode): J = int32 * jqg, jqg = jq * 2^jshift
    int jshift;            // float mode: bits the LDS sums are rounded off by when they go to HBM (0 in double)
    int nts;               // 1: the batch's particle state exceeds the last-level cache, so the
                           // particle kernels stream it with non-temporal loads and stores
    double cdep[3];        // Esirkepov factors -q w d_a / (dt dV) (times 1/jq in float mode)
    double cy2d;           // q w / dV (times 1/jq in float mode): J_y = cy2d * v_y * W_y in 2D
    double rho_c;          // q w / dV for the charge density
    int hz, hx, hy;        // stencil half-widths
    double tz[2][2 * PIC_MAX_HZ + 1];  // combined z taps: [0] Psi_E o filter, [1] Psi_B o filter
    double tx[2 * PIC_MAX_HX + 1];     // x filter taps
    double ty[2 * PIC_MAX_HX + 1];     // y filter taps (3D)
    // momentum-conserving gather (Eq. 5 scheme): the seen fields are written on
    // the integer nodes.  Along an axis where a component is half-staggered its
    // taps are those above composed with the two-point node average (tzn: Psi_B o
    // filter; txn, tyn: filter); the other taps are padded by one zero on each
    // side, and hz, hx, hy include the extra cell
    int nodal;
    double tzn[2 * PIC_MAX_HZ + 1];
    double txn[2 * PIC_MAX_HX + 1];
    double tyn[2 * PIC_MAX_HX + 1];
    // exact ratio variant: the transverse E are multiplied by Psi_E / Psi_B, the
    // denominator applied as Psi_B(S_z)^{-1} = rscale prod_q [(1 - l_q E^-1)(1 - l_q E)]^{-1}
    // along z (E = shift by one cell, one factor per real root of Psi_B)
    int ratio, nroot;
    double lam[8];
    double rscale;
    // grid planes (element type follows the precision)
    // E, B and J alternate between two sets of planes from step to step (index =
    // parity): the field kernels read one set with halos and write the other
    void *E[2][3], *B[2][3], *J[2][3];
    void *Et[3], *Bt[3];
    void *T1[6], *T2[6];   // intermediates of the separable seen-field passes
    double *rho0, *rho;
    // particles
    int *pidx;             // packed cell index: 2D x | z << 16, 3D x | y << 11 | z << 21
    void *poff[3];         // in-cell offsets in [0, 1) per active axis
    void *pu[3];           // momenta
    int *ppid;             // original particle number
    int *sidx, *spid, *srank, *stile;
    void *soff[3], *su[3];
    // tiles
    int *tstart;           // ntiles + 1 slot offsets
    int *tbox;             // per tile: lo[3] (wrapped cell coords), ext[3]
    int *tcount;
    int *flags;            // FLAG_*
    int *any_resort;       // one word shared by all instances: some instance set FLAG_RESORT
    // tiles whose particle box outgrew the LDS window, left by the particle kernel
    // for its global-memory pass (shared by all instances): [0] count, [1] blocks
    // of the pass that are done, then (instance, tile) pairs from [2]
    int *defer;
    double *diag;          // DG_*
    double *trace;         // trace_cap rows of 6 doubles
    // reverse mode (null unless gradient runs were planned)
    void *lE[3], *lB[3], *lJ[3], *lEt[3], *lBt[3];   // adjoint grid planes
    void *loff[3], *lu[3];                            // adjoint particle offsets / momenta
    double *grad;          // dW/dpsi_e[j]: PIC_GRAD_COPIES copies of 16 slots (j < 9), summed on the host
    double *loss;          // W
    int psi_deg, hzf;
    double tzf[2 * PIC_MAX_HZ + 1];  // z filter taps alone
    double sj[9][17];      // taps of S_z^j (half-width j), j <= psi_deg
    double cdep_r[3], cy2d_r;        // Esirkepov factors in real units (float mode unscaled)
    double psi_e[9];                 // Psi_E coefficients (1, 0, ... without the correction)
    // recording one tape slot (2D reverse sweep; null otherwise): the seen pass
    // also writes E1, B2 here, the particle kernel the state it starts from
    void *rE[3], *rB[3];
    int *rpidx, *rtbox;
    void *roff[3], *ru[3];
};

// gather schemes (template argument of the particle kernel)
enum {
    GATHER_GALERKIN = 0,   // Eq. 3: order l, lowered by one along half-staggered axes
    GATHER_UNIFORM = 1,    // Eq. 4: order l from each component's own Yee location
    GATHER_NODAL = 2       // Eq. 5: order l from the integer nodes (seen fields averaged there)
};

// Launch slot b -> tile in XCD-aware order: slot b runs on XCD b % 8, and each
// XCD gets a contiguous run of tiles (whose guard cells then share its L2)
__host__ __device__ inline int xcd_tile(int b, int nt)
{
    return (nt % 8 != 0) ? b : (b % 8) * (nt / 8) + b / 8;
}

// breakdown test of the correction polynomials (psi_setup.cpp)
bool psi_positive(const double *psi_e, const double *psi_b, int deg);
// real roots of a polynomial in s; -1 if one is not real (psi_setup.cpp)
int psi_real_roots(const double *coef, int deg, double *roots, double *lead);

// launch helpers implemented in pic_kernels.hip
struct LaunchCtx {
    const InstDesc *desc;       // device table
    hipStream_t stream;
    int dims, order, fp32;
    int yee_tz = 8, seen_tz = 16; // 2D field-kernel tile heights (x width 64)
    int waves4 = 0;               // 2D linear float particle kernel capped at 128 VGPRs
    int prefetch = 0;             // 2D linear float particle kernel loads one particle ahead
    // seen-stencil half-widths and Psi degree shared by every instance (-1: they differ)
    int hz = -1, hx = -1, hzf = -1, psi_deg = -1;
    const int *any_resort = nullptr;  // device word: a re-sort is pending
    const int *defer = nullptr;       // deferred-tile list (count, done count, pairs)
    int record = 0;                   // 2D: descriptors carry tape-recording pointers
    // parity of the current E, B (and of the J they were advanced with): the
    // Yee launch reads set par and writes set par ^ 1; every later launch of the
    // step is given the new parity
    int par = 0;
    int single = 0;                   // one instance: 2D field kernels take tile = block index
    int gather = GATHER_GALERKIN;     // gather scheme shared by every instance
    int ck = 0;                       // 2D Cole-Karkkainen curl in Faraday's law (every instance)
    int ratio = 0;                    // exact Psi_E / Psi_B on the transverse E (every instance)
    int inst0 = 0, ninst = 1;         // instances the launches cover (ratio solve grid)
    int rtiles = 0;                   // column tiles of the widest instance (ratio solve grid)
    int cus = 256;                    // compute units of the device
    int col_blocks[2] = {0, 0};       // 3D column passes (z, y): 256-thread blocks for the largest instance
    int x_blocks = 0;                 // 3D x pass: workgroups of 256 * PIC_SEEN_XSEG cells for the largest instance
    int defer_mode = -1;              // particle launch form: -1 by tile count, 0 inline, 1 deferring (2D)
};

int launch_yee(const LaunchCtx &c, const int2 *fwork, int nwork, const int2 *ywork, int nywork);
#define PIC_YEE_TX 64
int launch_seen(const LaunchCtx &c, const int2 *fwork, int nwork, const int2 *swork, int nswork);
// columns (one wave each) per workgroup of the Psi_B inversion along z, and its largest nz
#define PIC_RATIO_TC 4
#define PIC_RATIO_MAXNZ 1024
size_t seen_smem_bytes(int fp32, int tz, int hz, int hx);
int launch_particles(const LaunchCtx &c, const int2 *pwork, int nwork, int grid, int block,
                     const int wmax[3]);
size_t particle_smem_bytes(int dims, int fp32, const int wmax[3]);
// clear_any: the last re-sort launch of a step clears the shared pending word
int launch_resort(const LaunchCtx &c, const int2 *cwork, int ncwork, int n_inst_first, int n_inst, int clear_any);
// up to PIC_COPY_LIST device-to-device copies (16-byte aligned addresses,
// sizes a multiple of 4 bytes) in one launch
#define PIC_COPY_LIST 4
struct CopyList {
    const void *src[PIC_COPY_LIST];
    void *dst[PIC_COPY_LIST];
    long long bytes[PIC_COPY_LIST];
    int n = 0;
};
int launch_copy_list(hipStream_t st, const CopyList &L);
int launch_rho(const LaunchCtx &c, const int2 *pwork, int npwork, const int2 *fwork, int nfwork, const int wmax[3],
               int to_rho0);
int launch_diag(const LaunchCtx &c, const int2 *fwork, int nfwork, const int2 *pwork, int npwork, const int wmax[3]);
int launch_trace_rows(const LaunchCtx &c, const int2 *fwork, int nfwork, int *pos, double *trace, int n_inst,
                      int cap);
int launch_fill_bbox(const LaunchCtx &c, int inst_first, int n_inst);
size_t adjoint_smem_bytes(int dims, int fp32, const int wmax[3]);
int launch_adj_seed(const LaunchCtx &c, const int2 *fwork, int nfwork, const int2 *cwork, int ncwork);
size_t adj_seen_smem_bytes(int fp32);
// awork: 2D field tiles of 64 x 8 cells (PIC_ADJ_TZ rows) for the fused reverse kernels
#define PIC_ADJ_TZ 8
int launch_adj_step(const LaunchCtx &live, const LaunchCtx &tape, const int2 *fwork, int nfwork,
                    const int2 *swork, int nswork, const int2 *awork, int nawork, const int2 *pwork, int npwork,
                    int block, const int wmax[3]);
