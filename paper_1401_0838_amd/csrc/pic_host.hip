// Host side of the C ABI declared in include/pic_api.h: configuration checks,
// device arena layout, particle upload and tile sort, work lists, launch
// schedules (batched or per instance, eager or HIP-graph replay), and the
// accessors for fields, particles and diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "pic_api.h"
#include "pic_internal.h"
#include "pic_device.h"

namespace {

using pic::pack_cell;
using pic::unpack_cell;

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return fail(PIC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));               \
    } while (0)

struct Range { int off, n; };

// device copies of the state an adjoint run needs to restore or replay
struct Snap {
    void *E[3] = {nullptr, nullptr, nullptr}, *B[3] = {nullptr, nullptr, nullptr};
    void *J[3] = {nullptr, nullptr, nullptr};
    int *pidx = nullptr, *tbox = nullptr;
    void *poff[3] = {nullptr, nullptr, nullptr}, *pu[3] = {nullptr, nullptr, nullptr};
    void *Et[3] = {nullptr, nullptr, nullptr}, *Bt[3] = {nullptr, nullptr, nullptr};   // 2D tape slots
};

struct Layout {
    size_t bytes = 0;
    char *base = nullptr;
    template <class T> T *take(size_t count)
    {
        bytes = (bytes + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + bytes) : nullptr;
        bytes += count * sizeof(T);
        return p;
    }
};

int default_block() { return 256; }

// tile size and slack per axis for an instance
void tile_shape(const pic_config &c, int tile[3], int &slack)
{
    const int n[3] = {c.nx, c.dims == 3 ? c.ny : 1, c.nz};
    int def[3];
    if (c.dims == 2) {
        def[0] = 16; def[1] = 1; def[2] = 16;
        slack = 4;
    } else {
        // measured on the 128 x 128 x 256 cubic beam: 8 x 2 x 4 beat 4 x 4 x 4 by ~5 %
        def[0] = 8; def[1] = c.shape_order == 1 ? 4 : 2; def[2] = 4;
        slack = 2;
    }
    for (int a = 0; a < 3; a++) {
        int t = c.tile[a] > 0 ? c.tile[a] : def[a];
        if (c.dims == 2 && a == 1) t = 1;
        tile[a] = std::min(t, n[a]);
    }
}

// 2D default particle tiles are 16 x 16 cells.  When the whole batch has fewer
// than four such tiles per compute unit (1024), instances that leave the tile
// unset get 8 x 8 tiles so that the particle kernels still fill the chip.
std::vector<pic_config> resolve_tiles(const pic_config *cfgs, int n)
{
    std::vector<pic_config> v(cfgs, cfgs + n);
    if (n < 1 || v[0].dims != 2) return v;
    long long total = 0;
    for (const pic_config &c : v) {
        const int tx = c.tile[0] > 0 ? c.tile[0] : 16, tz = c.tile[2] > 0 ? c.tile[2] : 16;
        total += (long long)((c.nx + tx - 1) / tx) * ((c.nz + tz - 1) / tz);
    }
    if (total >= 1024) return v;
    for (pic_config &c : v)
        if (c.tile[0] <= 0 && c.tile[2] <= 0) { c.tile[0] = 8; c.tile[1] = 1; c.tile[2] = 8; }
    return v;
}

int validate(const pic_config &c, int idx)
{
    char buf[256];
    auto bad = [&](int code, const char *what) {
        snprintf(buf, sizeof buf, "instance %d: %s", idx, what);
        return fail(code, buf);
    };
    if (c.dims != 2 && c.dims != 3) return bad(PIC_EINVAL, "dims must be 2 or 3");
    if (c.nx < 1 || c.nz < 1 || c.ny < 1) return bad(PIC_EINVAL, "cell counts must be >= 1");
    if (c.dims == 2 && c.ny != 1) return bad(PIC_EINVAL, "ny must be 1 in 2D");
    if (c.dims == 2 && (c.nx > 65536 || c.nz > 65536)) return bad(PIC_EINVAL, "2D cell counts must be <= 65536");
    if (c.dims == 3 && (c.nx > 2048 || c.ny > 1024 || c.nz > 2048))
        return bad(PIC_EINVAL, "3D cell counts must be <= 2048 x 1024 x 2048 (packed int32 cell index)");
    if (!(c.dx > 0) || !(c.dz > 0) || (c.dims == 3 && !(c.dy > 0))) return bad(PIC_EINVAL, "cell sizes must be > 0");
    if (!(c.cdt > 0)) return bad(PIC_EINVAL, "c dt must be > 0");
    if (c.solver != PIC_YEE && c.solver != PIC_CK) return bad(PIC_EINVAL, "solver must be PIC_YEE or PIC_CK");
    if (c.solver == PIC_CK) {
        if (c.dims != 2) return bad(PIC_EUNSUPPORTED, "the Cole-Karkkainen solver is built for 2D");
        if (c.dx != c.dz) return bad(PIC_EUNSUPPORTED, "the Cole-Karkkainen solver needs square cells (dx == dz)");
        if (c.cdt >= c.dx) return bad(PIC_ECOURANT, "Cole-Karkkainen limit c dt < dx violated");
    } else {
        double s = 1.0 / (c.dx * c.dx) + 1.0 / (c.dz * c.dz) + (c.dims == 3 ? 1.0 / (c.dy * c.dy) : 0.0);
        if (c.cdt * std::sqrt(s) >= 1.0) return bad(PIC_ECOURANT, "Courant limit c dt < 1/sqrt(sum 1/d^2) violated");
    }
    if (c.shape_order != 1 && c.shape_order != 3) return bad(PIC_EINVAL, "shape_order must be 1 or 3");
    if (c.interp != PIC_GALERKIN && c.interp != PIC_UNIFORM && c.interp != PIC_MOMENTUM)
        return bad(PIC_EINVAL, "interp must be PIC_GALERKIN, PIC_UNIFORM or PIC_MOMENTUM");
    if (c.interp == PIC_MOMENTUM && c.adjoint_steps > 0)
        return bad(PIC_EUNSUPPORTED, "the reverse sweep is built for the Galerkin and Uniform gathers");
    if (c.precision != PIC_FP32 && c.precision != PIC_FP64) return bad(PIC_EINVAL, "precision");
    if (c.filter_npass < 0 || c.filter_npass > 8) return bad(PIC_EINVAL, "filter_npass must be in [0, 8]");
    // the node average of the momentum-conserving gather widens every stencil by one cell
    if (c.interp == PIC_MOMENTUM && c.filter_npass + 1 > PIC_MAX_HX)
        return bad(PIC_EINVAL, "filter_npass must be <= 7 with the momentum-conserving gather");
    if (c.correction != PIC_CORR_NONE && c.correction != PIC_CORR_SPLIT && c.correction != PIC_CORR_RATIO)
        return bad(PIC_EINVAL, "correction must be PIC_CORR_NONE, PIC_CORR_SPLIT or PIC_CORR_RATIO");
    if (c.correction == PIC_CORR_RATIO) {
        if (c.nz > PIC_RATIO_MAXNZ) return bad(PIC_EUNSUPPORTED, "the exact ratio needs nz <= 1024");
        if (c.adjoint_steps > 0) return bad(PIC_EUNSUPPORTED, "the reverse sweep needs the split correction");
        double roots[8], lead;
        if (c.psi_deg >= 1 && c.psi_deg <= 8) {
            const int nr = psi_real_roots(c.psi_b, c.psi_deg, roots, &lead);
            if (nr < 0) return bad(PIC_EUNSUPPORTED, "the exact ratio needs Psi_B with real roots only");
            for (int q = 0; q < nr; q++)
                if (roots[q] >= 0.0 && roots[q] <= 1.0) return bad(PIC_EPSI, "Psi_B has a root in [0, 1]");
        }
    }
    if (c.correction) {
        if (c.psi_deg < 1 || c.psi_deg > 8) return bad(PIC_EINVAL, "psi_deg must be in [1, 8]");
        if (c.psi_deg + c.filter_npass + (c.interp == PIC_MOMENTUM) > PIC_MAX_HZ)
            return bad(PIC_EINVAL, "z stencil too wide");
        if (!psi_positive(c.psi_e, c.psi_b, c.psi_deg))
            return bad(PIC_EPSI, "Psi_B <= 0 on s in [0,1] or Psi_E <= 0 on [0,1)");
    }
    if (!(c.m > 0) || !(c.weight >= 0) || !std::isfinite(c.q)) return bad(PIC_EINVAL, "species parameters");
    if (c.ion_mode != PIC_IONS_CHARGE && c.ion_mode != PIC_IONS_CHARGE_AND_CURRENT) return bad(PIC_EINVAL, "ion_mode");
    if (c.block != 0 && c.block != 256 && c.block != 512) return bad(PIC_EINVAL, "block must be 0, 256 or 512");
    if (c.trace_capacity < 0) return bad(PIC_EINVAL, "trace_capacity");
    if (c.adjoint_steps < 0 || (c.adjoint_steps > 0 && c.adjoint_ckpt < 1)) return bad(PIC_EINVAL, "adjoint sizes");
    return PIC_OK;
}

// polynomial (in the stencil algebra) convolution helpers: taps centred arrays
std::vector<double> conv(const std::vector<double> &a, const std::vector<double> &b)
{
    std::vector<double> r(a.size() + b.size() - 1, 0.0);
    for (size_t i = 0; i < a.size(); i++)
        for (size_t j = 0; j < b.size(); j++) r[i + j] += a[i] * b[j];
    return r;
}

// taps of Psi(S_z) with S_z = -(1/4)(1,-2,1): sum_j c_j S_z^j
std::vector<double> psi_taps(const double *c, int deg)
{
    const std::vector<double> S = {-0.25, 0.5, -0.25};
    std::vector<double> pw = {1.0};
    std::vector<double> acc(2 * deg + 1, 0.0);
    for (int j = 0; j <= deg; j++) {
        for (size_t t = 0; t < pw.size(); t++) acc[deg - j + t] += c[j] * pw[t];
        pw = conv(pw, S);
    }
    return acc;
}

std::vector<double> filter_taps(const pic_config &c)
{
    std::vector<double> t = {1.0};
    for (int k = 0; k < c.filter_npass; k++) {
        const double w = c.filter_w[k];
        t = conv(t, {w, 1.0 - 2.0 * w, w});
    }
    return t;
}

}  // namespace

struct pic_state {
    int n_inst = 0, dims = 2, order = 1, fp32 = 1;
    int gather = GATHER_GALERKIN;    // gather scheme of every instance
    int ck = 0;                      // Cole-Karkkainen solver (every instance)
    int ratio = 0;                   // exact Psi_E / Psi_B on the transverse E (every instance)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int static_dev = -1;             // device whose static arena holds this state (pic_init_static)
    char *arena = nullptr;
    size_t arena_bytes = 0;
    std::vector<pic_config> cfg;
    std::vector<InstDesc> desc;
    std::vector<int64_t> np;
    InstDesc *d_desc = nullptr;
    int2 *fwork = nullptr, *pwork = nullptr, *cwork = nullptr, *swork = nullptr, *ywork = nullptr, *awork = nullptr;
    int nfwork = 0, npwork = 0, ncwork = 0, nswork = 0, nywork = 0, nawork = 0;
    std::vector<Range> frange, prange, crange, srange, yrange;
    int wmax[3] = {1, 1, 1};
    int block = 256;
    int sched = PIC_SCHED_BATCHED, use_graph = 1;
    int graph_k = 16;                // steps per captured graph (and re-sort period)
    int yee_tz = 8, seen_tz = 16;    // 2D field-kernel tile heights (tunable)
    int waves4 = 0;                  // particle kernel capped at four waves per SIMD (tunable)
    int prefetch = 0;                // particle kernel loads one particle ahead (tunable)
    // captured step graphs keyed by (steps, re-sort check at the end, parity of
    // the state they start from); a pic_step call replays at most three kinds:
    // a head up to the next re-sort point, whole periods, and a tail
    std::map<std::tuple<int, int, int>, hipGraphExec_t> gexec;
    int parity = 0;                  // which set of E, B, J planes is current
    long long step = 0;
    int *trace_pos = nullptr;
    int *any_resort = nullptr;       // device word shared by all instances: a re-sort is pending
    int *defer = nullptr;            // deferred-tile list of the particle kernel (InstDesc::defer)
    int cus = 256;                   // compute units of the device
    int defer_mode = -1;             // particle launch form: -1 by tile count, 0 inline, 1 deferring (2D)
    double *trace = nullptr;
    int trace_cap = 0;
    // reverse mode
    int adj_steps = 0, adj_k = 0;
    bool no_resort = false;
    int adj_pending = 0;                         // steps of the last pic_adjoint_forward
    hipGraphExec_t gexec_adj_fwd[2] = {nullptr, nullptr}, gexec_adj_seg = nullptr;
    std::vector<std::vector<Snap>> ckpt, tape;   // [instance][slot]
    int adj_slots = 0;                           // tape slots: adj_k, two banks of adj_k in 2D
    // 2D reverse sweep in two streams: a segment is recomputed (main stream)
    // into one tape bank while the previous one is reversed (rstream) from the other
    hipStream_t rstream = nullptr;
    hipEvent_t ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr}, ev_join = nullptr;
    hipGraphExec_t gexec_adj_rec[2] = {nullptr, nullptr}, gexec_adj_rev[2] = {nullptr, nullptr};
    InstDesc *d_tape_desc = nullptr;             // adj_slots * n_inst descriptors
    InstDesc *d_rec_desc = nullptr;              // 2D: the live step recording into tape slot k
    int adj_wmax[3] = {1, 1, 1};
};

namespace {

LaunchCtx ctx(const pic_state *s)
{
    LaunchCtx c;
    c.desc = s->d_desc;
    c.stream = s->stream;
    c.dims = s->dims;
    c.order = s->order;
    c.fp32 = s->fp32;
    c.yee_tz = s->yee_tz;
    c.seen_tz = s->seen_tz;
    c.waves4 = s->waves4;
    c.prefetch = s->prefetch;
    c.any_resort = s->any_resort;
    c.defer = s->defer;
    c.cus = s->cus;
    c.defer_mode = s->defer_mode;
    c.par = s->parity;
    c.single = s->n_inst == 1;
    c.gather = s->gather;
    c.ck = s->ck;
    c.ninst = s->n_inst;
    c.ratio = s->ratio;
    for (const InstDesc &d : s->desc) {
        c.rtiles = std::max(c.rtiles, (d.n[0] * d.n[1] + PIC_RATIO_TC - 1) / PIC_RATIO_TC);
        // 3D column passes: one thread per column and run of PIC_COL_RUN cells
        const long long tz = (long long)d.n[0] * d.n[1] * ((d.n[2] + PIC_COL_RUN - 1) / PIC_COL_RUN);
        const long long ty = (long long)d.n[0] * d.n[2] * ((d.n[1] + PIC_COL_RUN - 1) / PIC_COL_RUN);
        c.col_blocks[0] = std::max(c.col_blocks[0], (int)((tz + 255) / 256));
        c.col_blocks[1] = std::max(c.col_blocks[1], (int)((ty + 255) / 256));
        c.x_blocks = std::max(c.x_blocks, (int)((d.ncell + 256 * PIC_SEEN_XSEG - 1) / (256 * PIC_SEEN_XSEG)));
    }
    if (!s->desc.empty()) {
        const InstDesc &d0 = s->desc[0];
        c.hz = d0.hz; c.hx = d0.hx; c.hzf = d0.hzf; c.psi_deg = d0.psi_deg;
        for (const InstDesc &d : s->desc)
            if (d.hz != d0.hz || d.hx != d0.hx || d.hzf != d0.hzf || d.psi_deg != d0.psi_deg) {
                c.hz = c.hx = c.hzf = c.psi_deg = -1;
                break;
            }
    }
    return c;
}

int yee_tz_eff(int tz, int fp32) { return (!fp32 && tz > 8) ? 8 : tz; }
// 2D seen-field tile height: 32 rows of doubles with the widest stencils exceed
// 64 KB of LDS; the 128-row streamed segments are built for float and the usual
// stencil widths (half-widths hz, hx common to the batch, -1 if they differ)
int seen_tz_eff(int tz, int fp32, int hz, int hx)
{
    if (tz == 128 && !(fp32 && ((hz == 8 && hx == 4) || (hz == 9 && hx == 5)))) tz = 32;
    return (!fp32 && tz > 16) ? 16 : tz;
}

// tape slots of the reverse sweep: one segment's steps, twice in 2D (two banks)
int tape_slots(const pic_config &c) { return (c.dims == 2 ? 2 : 1) * c.adjoint_ckpt; }

// Lay out all arrays; with base == nullptr only the size is computed.
size_t layout(pic_state *s, const pic_config *cfgs, int n_inst, const int64_t *np, char *base)
{
    Layout L;
    L.base = base;
    const size_t R = cfgs[0].precision == PIC_FP32 ? 4 : 8;
    // current planes: 32-bit fixed point in float mode, double otherwise
    const size_t JB = cfgs[0].precision == PIC_FP32 ? 4 : 8;
    InstDesc *dd = L.take<InstDesc>(n_inst);
    if (s) s->d_desc = dd;
    size_t nf = 0, npw = 0, nc = 0, ns = 0, ny = 0;
    std::vector<int> ntiles(n_inst);
    for (int i = 0; i < n_inst; i++) {
        const pic_config &c = cfgs[i];
        const size_t ncell = (size_t)c.nx * c.ny * c.nz;
        int tile[3], slack;
        tile_shape(c, tile, slack);
        const int nt = ((c.nx + tile[0] - 1) / tile[0]) * ((c.ny + tile[1] - 1) / tile[1]) *
                       ((c.nz + tile[2] - 1) / tile[2]);
        ntiles[i] = nt;
        nf += (ncell + PIC_FIELD_CHUNK - 1) / PIC_FIELD_CHUNK;
        // sized for the smallest selectable tiles (seen 8 rows, Yee 4 rows)
        ns += (size_t)((c.nx + PIC_SEEN_TX - 1) / PIC_SEEN_TX) * ((c.nz + 8 - 1) / 8);
        ny += (size_t)((c.nx + PIC_YEE_TX - 1) / PIC_YEE_TX) * ((c.nz + 4 - 1) / 4);
        npw += nt;
        nc += (np[i] + PIC_PART_CHUNK - 1) / PIC_PART_CHUNK;
    }
    int2 *fw = L.take<int2>(nf), *pw = L.take<int2>(npw), *cw = L.take<int2>(std::max<size_t>(nc, 1));
    int2 *sw = L.take<int2>(ns), *yw = L.take<int2>(ny), *aw = L.take<int2>(ns);
    if (s) { s->fwork = fw; s->pwork = pw; s->cwork = cw; s->swork = sw; s->ywork = yw; s->awork = aw; }
    int *tpos = L.take<int>(64);
    if (s) s->trace_pos = tpos;
    int *anyr = L.take<int>(64);
    if (s) s->any_resort = anyr;
    int *defer = L.take<int>(2 + 2 * std::max<size_t>(npw, 1));
    if (s) s->defer = defer;
    int cap = 0;
    for (int i = 0; i < n_inst; i++) cap = std::max(cap, cfgs[i].trace_capacity);
    // one spare row: each step clears the row the next step writes, so a ring
    // of cap + 1 rows always holds the last cap complete rows
    double *tr = L.take<double>((size_t)(std::max(cap, 1) + 1) * n_inst * 6);
    if (s) { s->trace = tr; s->trace_cap = cap > 0 ? cap + 1 : 0; }
    if (cfgs[0].adjoint_steps > 0) {
        const int nslot = tape_slots(cfgs[0]);
        InstDesc *td = L.take<InstDesc>((size_t)nslot * n_inst);
        if (s) s->d_tape_desc = td;
        InstDesc *rd = L.take<InstDesc>((size_t)nslot * n_inst);
        if (s) s->d_rec_desc = rd;
    }
    for (int i = 0; i < n_inst; i++) {
        const pic_config &c = cfgs[i];
        const size_t ncell = (size_t)c.nx * c.ny * c.nz;
        const size_t n = (size_t)np[i];
        InstDesc *D = s ? &s->desc[i] : nullptr;
        auto plane = [&](size_t bytes_per) { return (void *)L.take<char>(ncell * bytes_per); };
        // E, B and J each occupy one contiguous region (planes in component
        // order) so that checkpoints copy them with one transfer each
        void *pe[2][3], *pb[2][3], *pj[2][3], *pet[3], *pbt[3];
        for (int q = 0; q < 2; q++) {
            for (int k = 0; k < 3; k++) pe[q][k] = plane(R);
            for (int k = 0; k < 3; k++) pb[q][k] = plane(R);
            for (int k = 0; k < 3; k++) pj[q][k] = plane(JB);
        }
        for (int k = 0; k < 3; k++) pet[k] = plane(R);
        for (int k = 0; k < 3; k++) pbt[k] = plane(R);
        if (D)
            for (int k = 0; k < 3; k++) {
                for (int q = 0; q < 2; q++) { D->E[q][k] = pe[q][k]; D->B[q][k] = pb[q][k]; D->J[q][k] = pj[q][k]; }
                D->Et[k] = pet[k];
                D->Bt[k] = pbt[k];
            }
        const bool adj = c.adjoint_steps > 0;
        for (int k = 0; k < 6; k++) {
            void *t1 = plane(R);
            void *t2 = c.dims == 3 ? plane(R) : nullptr;
            if (D) { D->T1[k] = t1; D->T2[k] = t2; }
        }
        double *r0 = L.take<double>(ncell), *r1 = L.take<double>(ncell);
        // particle state (cell index, offsets, momenta) is one contiguous region
        int *pidx = L.take<int>(n);
        void *poff[3] = {nullptr, nullptr, nullptr}, *pu[3], *soff[3] = {nullptr, nullptr, nullptr}, *su[3];
        for (int a = 0; a < 3; a++)
            if (!(c.dims == 2 && a == 1)) poff[a] = L.take<char>(n * R);
        for (int a = 0; a < 3; a++) pu[a] = L.take<char>(n * R);
        int *ppid = L.take<int>(n);
        int *sidx = L.take<int>(n), *spid = L.take<int>(n), *srank = L.take<int>(n), *stile = L.take<int>(n);
        for (int a = 0; a < 3; a++) {
            if (!(c.dims == 2 && a == 1)) soff[a] = L.take<char>(n * R);
            su[a] = L.take<char>(n * R);
        }
        int *tstart = L.take<int>(ntiles[i] + 1), *tbox = L.take<int>((size_t)ntiles[i] * 6);
        int *tcount = L.take<int>(ntiles[i]);
        int *flags = L.take<int>(FLAG_COUNT);
        double *diag = L.take<double>(DG_COUNT);
        if (adj) {
            const int K = c.adjoint_ckpt;
            const int nck = (c.adjoint_steps + K - 1) / K + 1;
            for (int k = 0; k < 3; k++) {
                void *a = plane(R), *b = plane(R), *j = plane(R), *e = plane(R), *f = plane(R);
                if (D) { D->lE[k] = a; D->lB[k] = b; D->lJ[k] = j; D->lEt[k] = e; D->lBt[k] = f; }
            }
            for (int a = 0; a < 3; a++) {
                void *lo = (c.dims == 2 && a == 1) ? nullptr : (void *)L.take<char>(n * R);
                void *lu = L.take<char>(n * R);
                if (D) { D->loff[a] = lo; D->lu[a] = lu; }
            }
            double *g = L.take<double>(16 * PIC_GRAD_COPIES);
            if (D) { D->grad = g; D->loss = g + 9; }
            // same region order as the live arrays (see above)
            auto snap = [&](bool with_j, bool with_seen) {
                Snap sn;
                for (int k = 0; k < 3; k++) sn.E[k] = plane(R);
                for (int k = 0; k < 3; k++) sn.B[k] = plane(R);
                if (with_j)
                    for (int k = 0; k < 3; k++) sn.J[k] = plane(JB);
                sn.pidx = L.take<int>(n);
                for (int a = 0; a < 3; a++)
                    if (!(c.dims == 2 && a == 1)) sn.poff[a] = L.take<char>(n * R);
                for (int a = 0; a < 3; a++) sn.pu[a] = L.take<char>(n * R);
                sn.tbox = L.take<int>((size_t)ntiles[i] * 6);
                if (with_seen)
                    for (int k = 0; k < 3; k++) { sn.Et[k] = plane(R); sn.Bt[k] = plane(R); }
                return sn;
            };
            std::vector<Snap> ck, tp;
            for (int k = 0; k < nck; k++) ck.push_back(snap(true, false));
            for (int k = 0; k < tape_slots(c); k++) tp.push_back(snap(false, c.dims == 2));
            if (s) { s->ckpt.push_back(ck); s->tape.push_back(tp); }
        }
        if (D) {
            D->rho0 = r0; D->rho = r1;
            D->pidx = pidx; D->ppid = ppid; D->sidx = sidx; D->spid = spid; D->srank = srank; D->stile = stile;
            for (int a = 0; a < 3; a++) { D->poff[a] = poff[a]; D->pu[a] = pu[a]; D->soff[a] = soff[a]; D->su[a] = su[a]; }
            D->tstart = tstart; D->tbox = tbox; D->tcount = tcount; D->flags = flags; D->diag = diag;
            D->trace = tr;
        }
    }
    return L.bytes + 256;
}

void fill_desc(InstDesc &D, const pic_config &c, const pic_particles &p)
{
    const bool f32 = c.precision == PIC_FP32;
    D.n[0] = c.nx; D.n[1] = c.dims == 3 ? c.ny : 1; D.n[2] = c.nz;
    D.ncell = D.n[0] * D.n[1] * D.n[2];
    int slack;
    tile_shape(c, D.tile, slack);
    for (int a = 0; a < 3; a++) D.nt[a] = (D.n[a] + D.tile[a] - 1) / D.tile[a];
    D.ntiles = D.nt[0] * D.nt[1] * D.nt[2];
    D.trace_cap = c.trace_capacity;
    D.np = p.n;
    D.d[0] = c.dx; D.d[1] = c.dims == 3 ? c.dy : 1.0; D.d[2] = c.dz;
    D.dt = c.cdt;
    for (int a = 0; a < 3; a++) D.dtd[a] = c.cdt / D.d[a];
    D.qdt2m = c.q * c.cdt / (2.0 * c.m);
    D.w = c.weight;
    D.m = c.m;
    D.dV = c.dims == 3 ? c.dx * c.dy * c.dz : c.dx * c.dz;
    const double qw = c.q * c.weight;
    // fixed-point quantum: 2^-28 of the largest single-particle contribution scale
    double U = std::fabs(qw) / D.dV;
    for (int a = 0; a < 3; a++) U = std::max(U, std::fabs(qw) * D.d[a] / (c.cdt * D.dV));
    D.jq = (f32 && U > 0) ? U * std::ldexp(1.0, -28) : 1.0;
    // HBM planes (float mode): the quantum is about 2^-21 of the current a
    // beam moving at c carries through the densest cell of the initial load,
    // J_s = kmax |q w| / dV, so a current word holds at least 2^9 J_s inside the
    // checked range +-2^30 (beyond it the instance is flagged); a tile's LDS sum
    // is rounded to it once per step
    D.jshift = 0;
    if (f32 && U > 0) {
        std::vector<int> cnt((size_t)D.ncell, 0);
        int kmax = 0;
        for (int64_t i = 0; i < p.n; i++) {
            long long cell = 0;
            for (int a = 2; a >= 0; a--) {
                if (c.dims == 2 && a == 1) continue;
                long long ci = (long long)std::floor(p.pos[a][i] / D.d[a]) % D.n[a];
                ci += ci < 0 ? D.n[a] : 0;
                cell = cell * D.n[a] + ci;
            }
            kmax = std::max(kmax, ++cnt[(size_t)cell]);
        }
        const double js = kmax * std::fabs(qw) / D.dV;
        if (js > 0) D.jshift = std::min(24, std::max(0, (int)std::floor(std::log2(js / U * 128.0))));
    }
    D.jqg = D.jq * std::ldexp(1.0, D.jshift);
    const double sc = f32 ? 1.0 / D.jq : 1.0;
    for (int a = 0; a < 3; a++) D.cdep[a] = -qw * D.d[a] / (c.cdt * D.dV) * sc;
    D.cy2d = qw / D.dV * sc;
    D.rho_c = qw / D.dV;
    // uniform ion current: minus the initial mean beam current
    double sv[3] = {0, 0, 0};
    if (c.ion_mode == PIC_IONS_CHARGE_AND_CURRENT) {
        for (int64_t i = 0; i < p.n; i++) {
            const double ux = p.mom[0][i], uy = p.mom[1][i], uz = p.mom[2][i];
            const double ig = 1.0 / std::sqrt(1.0 + ux * ux + uy * uy + uz * uz);
            sv[0] += ux * ig; sv[1] += uy * ig; sv[2] += uz * ig;
        }
    }
    for (int a = 0; a < 3; a++) D.jbg[a] = -qw * sv[a] / ((double)D.ncell * D.dV);
    // seen-field stencils
    const std::vector<double> fz = filter_taps(c);
    std::vector<double> ze = fz, zb = fz;
    if (c.correction) {
        ze = conv(psi_taps(c.psi_e, c.psi_deg), fz);
        zb = conv(psi_taps(c.psi_b, c.psi_deg), fz);
    }
    D.ratio = c.correction == PIC_CORR_RATIO;
    D.nroot = 0;
    D.rscale = 1.0;
    std::memset(D.lam, 0, sizeof D.lam);
    if (D.ratio) {
        // E_z and B are filtered only; the transverse E get Psi_E here and
        // Psi_B(S_z)^{-1} after the seen pass, one (S_z - r) factor per root:
        // (S_z - r) y = x  <=>  (1 - l E^-1)(1 - l E) y = 4 l x,  l + 1/l = 2 - 4 r
        zb.assign(ze.size(), 0.0);
        const size_t off = (ze.size() - fz.size()) / 2;
        for (size_t t = 0; t < fz.size(); t++) zb[off + t] = fz[t];
        double roots[8], lead;
        D.nroot = psi_real_roots(c.psi_b, c.psi_deg, roots, &lead);
        D.rscale = 1.0 / lead;
        for (int q = 0; q < D.nroot; q++) {
            const double cq = 2.0 - 4.0 * roots[q];
            const double l = 0.5 * cq - std::copysign(std::sqrt(0.25 * cq * cq - 1.0), cq);
            D.lam[q] = l;
            D.rscale *= 4.0 * l;
        }
    }
    D.hz = (int)(ze.size() / 2);
    D.hx = (int)(fz.size() / 2);
    D.hy = c.dims == 3 ? D.hx : 0;
    std::memset(D.tz, 0, sizeof D.tz);
    std::memset(D.tx, 0, sizeof D.tx);
    std::memset(D.ty, 0, sizeof D.ty);
    std::memset(D.tzn, 0, sizeof D.tzn);
    std::memset(D.txn, 0, sizeof D.txn);
    std::memset(D.tyn, 0, sizeof D.tyn);
    D.nodal = c.interp == PIC_MOMENTUM;
    if (D.nodal) {
        // fields seen on the integer nodes: node n of a component half-staggered
        // along an axis is the mean of its samples at n - 1/2 and n + 1/2 (array
        // slots n - 1 and n), i.e. the taps composed with (1/2 at -1, 1/2 at 0);
        // every stencil grows by one cell (zero-padded where not staggered)
        const std::vector<double> avg = {0.5, 0.5, 0.0};
        const std::vector<double> pad = {0.0, 1.0, 0.0};
        const std::vector<double> zn = conv(zb, avg), fn = conv(fz, avg);
        ze = conv(ze, pad);
        zb = conv(zb, pad);
        const std::vector<double> fp = conv(fz, pad);
        D.hz = (int)(ze.size() / 2);
        D.hx = (int)(fp.size() / 2);
        D.hy = c.dims == 3 ? D.hx : 0;
        for (size_t t = 0; t < zn.size(); t++) D.tzn[t] = zn[t];
        for (size_t t = 0; t < fn.size(); t++) { D.txn[t] = fn[t]; D.tyn[t] = fn[t]; }
        for (size_t t = 0; t < fp.size(); t++) { D.tx[t] = fp[t]; D.ty[t] = fp[t]; }
    } else {
        for (size_t t = 0; t < fz.size(); t++) { D.tx[t] = fz[t]; D.ty[t] = fz[t]; }
    }
    for (size_t t = 0; t < ze.size(); t++) { D.tz[0][t] = ze[t]; D.tz[1][t] = zb[t]; }
    // reverse mode: filter-only z taps, taps of S_z^j, unscaled deposit factors
    std::memset(D.tzf, 0, sizeof D.tzf);
    D.hzf = (int)(fz.size() / 2);
    for (size_t t = 0; t < fz.size(); t++) D.tzf[t] = fz[t];
    D.psi_deg = c.correction ? c.psi_deg : 0;
    std::memset(D.sj, 0, sizeof D.sj);
    std::vector<double> pw = {1.0};
    for (int j = 0; j <= 8; j++) {
        for (size_t t = 0; t < pw.size(); t++) D.sj[j][8 - j + t] = pw[t];
        pw = conv(pw, {-0.25, 0.5, -0.25});
    }
    for (int a = 0; a < 3; a++) D.cdep_r[a] = -qw * D.d[a] / (c.cdt * D.dV);
    D.cy2d_r = qw / D.dV;
    for (int j = 0; j < 9; j++) D.psi_e[j] = c.correction ? (j <= c.psi_deg ? c.psi_e[j] : 0.0) : (j == 0 ? 1.0 : 0.0);
}

template <class R>
int upload_particles(pic_state *s, int inst, const pic_particles &p)
{
    const InstDesc &D = s->desc[inst];
    const int dims = s->dims;
    const int64_t n = p.n;
    std::vector<int> cell(n), tile(n), rank(n);
    std::vector<unsigned> packed(n);
    std::vector<R> off[3];
    for (int a = 0; a < 3; a++) off[a].resize(dims == 2 && a == 1 ? 0 : n);
    for (int64_t i = 0; i < n; i++) {
        int c[3] = {0, 0, 0};
        for (int a = 0; a < 3; a++) {
            if (dims == 2 && a == 1) continue;
            const double x = p.pos[a][i] / D.d[a];
            double f = std::floor(x);
            double o = x - f;
            long long ci = (long long)f;
            R ro = (R)o;
            if (ro >= R(1)) { ro = R(0); ci += 1; }
            ci %= D.n[a];
            if (ci < 0) ci += D.n[a];
            c[a] = (int)ci;
            off[a][i] = ro;
        }
        cell[i] = (c[2] * D.n[1] + c[1]) * D.n[0] + c[0];
        packed[i] = dims == 2 ? pack_cell<2>(c[0], c[1], c[2]) : pack_cell<3>(c[0], c[1], c[2]);
        tile[i] = ((c[2] / D.tile[2]) * D.nt[1] + c[1] / D.tile[1]) * D.nt[0] + c[0] / D.tile[0];
    }
    // order: by tile, then by rank within the cell, then by cell, so that
    // consecutive lanes of a wavefront work on different cells
    std::vector<int> cnt(D.ncell, 0);
    int kmax = 0;
    for (int64_t i = 0; i < n; i++) { rank[i] = cnt[cell[i]]++; kmax = std::max(kmax, rank[i] + 1); }
    std::vector<int64_t> order(n), tmp(n);
    {   // stable counting sort by cell
        std::vector<int64_t> off_c(D.ncell + 1, 0);
        for (int64_t i = 0; i < n; i++) off_c[cell[i] + 1]++;
        for (int c = 0; c < D.ncell; c++) off_c[c + 1] += off_c[c];
        for (int64_t i = 0; i < n; i++) order[off_c[cell[i]]++] = i;
    }
    {   // stable by rank
        std::vector<int64_t> off_k(kmax + 1, 0);
        for (int64_t i = 0; i < n; i++) off_k[rank[i] + 1]++;
        for (int k = 0; k < kmax; k++) off_k[k + 1] += off_k[k];
        for (int64_t j = 0; j < n; j++) { int64_t i = order[j]; tmp[off_k[rank[i]]++] = i; }
    }
    std::vector<int> tstart(D.ntiles + 1, 0);
    {   // stable by tile
        for (int64_t i = 0; i < n; i++) tstart[tile[i] + 1]++;
        for (int t = 0; t < D.ntiles; t++) tstart[t + 1] += tstart[t];
        std::vector<int> fill(tstart.begin(), tstart.end() - 1);
        for (int64_t j = 0; j < n; j++) { int64_t i = tmp[j]; order[fill[tile[i]]++] = i; }
    }
    std::vector<int> h_idx(n), h_pid(n);
    std::vector<R> h_off[3], h_u[3];
    for (int a = 0; a < 3; a++) {
        if (!(dims == 2 && a == 1)) h_off[a].resize(n);
        h_u[a].resize(n);
    }
    for (int64_t j = 0; j < n; j++) {
        const int64_t i = order[j];
        h_idx[j] = (int)packed[i];
        h_pid[j] = (int)i;
        for (int a = 0; a < 3; a++) {
            if (!(dims == 2 && a == 1)) h_off[a][j] = off[a][i];
            h_u[a][j] = (R)p.mom[a][i];
        }
    }
    hipStream_t st = s->stream;
    HIP_TRY(hipMemcpyAsync(D.pidx, h_idx.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(D.ppid, h_pid.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
    for (int a = 0; a < 3; a++) {
        if (!(dims == 2 && a == 1))
            HIP_TRY(hipMemcpyAsync(D.poff[a], h_off[a].data(), n * sizeof(R), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(D.pu[a], h_u[a].data(), n * sizeof(R), hipMemcpyHostToDevice, st));
    }
    HIP_TRY(hipMemcpyAsync(D.tstart, tstart.data(), tstart.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // host vectors go out of scope
    return PIC_OK;
}

// bytes of the contiguous regions [E..B], [J], [cell index..momenta]
size_t region_fields(const InstDesc &D, size_t R)
{
    return (size_t)((char *)D.B[0][2] - (char *)D.E[0][0]) + D.ncell * R;
}
size_t region_j(const InstDesc &D, size_t jb)
{
    return (size_t)((char *)D.J[0][2] - (char *)D.J[0][0]) + (size_t)D.ncell * jb;
}
size_t region_particles(const InstDesc &D, size_t R)
{
    return (size_t)((char *)D.pu[2] - (char *)D.pidx) + (size_t)D.np * R;
}

// particle state and tile boxes of one instance to (save) or from a snapshot
int snap_copy_particles(pic_state *s, int inst, const Snap &sn, bool save)
{
    const InstDesc &D = s->desc[inst];
    const size_t R = s->fp32 ? 4 : 8;
    const hipMemcpyKind kd = hipMemcpyDeviceToDevice;
    auto cp = [&](void *live, void *snapp, size_t bytes) {
        if (!bytes || !live || !snapp) return hipSuccess;
        return save ? hipMemcpyAsync(snapp, live, bytes, kd, s->stream) : hipMemcpyAsync(live, snapp, bytes, kd, s->stream);
    };
    if (D.np > 0) HIP_TRY(cp(D.pidx, sn.pidx, region_particles(D, R)));
    HIP_TRY(cp(D.tbox, sn.tbox, (size_t)D.ntiles * 6 * 4));
    return PIC_OK;
}

// E and B (set q) of one instance into a snapshot
int snap_copy_fields(pic_state *s, int inst, const Snap &sn, int q)
{
    const InstDesc &D = s->desc[inst];
    HIP_TRY(hipMemcpyAsync(sn.E[0], D.E[q][0], region_fields(D, s->fp32 ? 4 : 8), hipMemcpyDeviceToDevice,
                           s->stream));
    return PIC_OK;
}

// XCD-aware order of one instance's tiles: launch slot b runs on XCD b % 8,
// so give each XCD a contiguous run of tiles (their halos share that XCD's L2)
void tile_order(int nt, std::vector<int> &out)
{
    out.resize(nt);
    if (nt % 8 != 0) {
        for (int t = 0; t < nt; t++) out[t] = t;
        return;
    }
    for (int b = 0; b < nt; b++) out[b] = xcd_tile(b, nt);
}

int build_worklists(pic_state *s)
{
    std::vector<int2> fw, pw, cw, sw, yw, aw;
    s->frange.clear(); s->prange.clear(); s->crange.clear(); s->srange.clear(); s->yrange.clear();
    const int ytz = yee_tz_eff(s->yee_tz, s->fp32), stz = s->seen_tz;
    std::vector<int> ord;
    for (int i = 0; i < s->n_inst; i++) {
        const InstDesc &D = s->desc[i];
        Range r{(int)fw.size(), 0};
        for (int k = 0; k < (D.ncell + PIC_FIELD_CHUNK - 1) / PIC_FIELD_CHUNK; k++) fw.push_back(make_int2(i, k));
        r.n = (int)fw.size() - r.off;
        s->frange.push_back(r);
        Range q{(int)pw.size(), 0};
        tile_order(D.ntiles, ord);
        for (int t = 0; t < D.ntiles; t++) pw.push_back(make_int2(i, ord[t]));
        q.n = (int)pw.size() - q.off;
        s->prange.push_back(q);
        // the 2D field tiles in the same XCD-aware order as the particle tiles:
        // each XCD takes a contiguous run of rows of tiles, so the halo rows a
        // tile shares with its neighbour along z are read into one L2
        Range sr{(int)sw.size(), 0};
        // (the streamed pass, seen_tz 128, takes strips PIC_SEEN_SW columns wide)
        const int stw = stz == 128 ? PIC_SEEN_SW : PIC_SEEN_TX;
        const int nst = ((D.n[0] + stw - 1) / stw) * ((D.n[2] + stz - 1) / stz);
        tile_order(nst, ord);
        for (int k = 0; k < nst; k++) sw.push_back(make_int2(i, ord[k]));
        sr.n = (int)sw.size() - sr.off;
        s->srange.push_back(sr);
        Range yr{(int)yw.size(), 0};
        const int nyt = ((D.n[0] + PIC_YEE_TX - 1) / PIC_YEE_TX) * ((D.n[2] + ytz - 1) / ytz);
        tile_order(nyt, ord);
        for (int k = 0; k < nyt; k++) yw.push_back(make_int2(i, ord[k]));
        yr.n = (int)yw.size() - yr.off;
        s->yrange.push_back(yr);
        const int nat = ((D.n[0] + PIC_SEEN_TX - 1) / PIC_SEEN_TX) * ((D.n[2] + PIC_ADJ_TZ - 1) / PIC_ADJ_TZ);
        for (int k = 0; k < nat; k++) aw.push_back(make_int2(i, k));
        Range c{(int)cw.size(), 0};
        for (long long k = 0; k < (D.np + PIC_PART_CHUNK - 1) / PIC_PART_CHUNK; k++) cw.push_back(make_int2(i, (int)k));
        c.n = (int)cw.size() - c.off;
        s->crange.push_back(c);
    }
    s->nfwork = (int)fw.size();
    s->npwork = (int)pw.size();
    s->ncwork = (int)cw.size();
    s->nswork = (int)sw.size();
    s->nywork = (int)yw.size();
    s->nawork = (int)aw.size();
    HIP_TRY(hipMemcpyAsync(s->awork, aw.data(), aw.size() * sizeof(int2), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->ywork, yw.data(), yw.size() * sizeof(int2), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->swork, sw.data(), sw.size() * sizeof(int2), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->fwork, fw.data(), fw.size() * sizeof(int2), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->pwork, pw.data(), pw.size() * sizeof(int2), hipMemcpyHostToDevice, s->stream));
    if (!cw.empty())
        HIP_TRY(hipMemcpyAsync(s->cwork, cw.data(), cw.size() * sizeof(int2), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return PIC_OK;
}

// one step's launches for instances [i0, i0 + ni) using the given work ranges
// one step's launches; the Yee launch reads the current parity, the rest see the new one
int enqueue_step_range(pic_state *s, const Range &f, const Range &sr, const Range &yr, const Range &p, int i0,
                       int ni)
{
    LaunchCtx c = ctx(s);
    c.inst0 = i0;
    c.ninst = ni;
    if (launch_yee(c, s->fwork + f.off, f.n, s->ywork + yr.off, yr.n)) return fail(PIC_EHIP, "yee launch");
    c.par ^= 1;
    if (launch_seen(c, s->fwork + f.off, f.n, s->swork + sr.off, sr.n)) return fail(PIC_EHIP, "seen launch");
    if (launch_particles(c, s->pwork + p.off, p.n, 0, s->block, s->wmax)) return fail(PIC_EHIP, "particle launch");
    return PIC_OK;
}

int enqueue_step(pic_state *s)
{
    if (s->sched == PIC_SCHED_BATCHED) {
        int rc = enqueue_step_range(s, Range{0, s->nfwork}, Range{0, s->nswork}, Range{0, s->nywork},
                                    Range{0, s->npwork}, 0, s->n_inst);
        if (rc) return rc;
    } else {
        for (int i = 0; i < s->n_inst; i++) {
            int rc = enqueue_step_range(s, s->frange[i], s->srange[i], s->yrange[i], s->prange[i], i, 1);
            if (rc) return rc;
        }
    }
    s->parity ^= 1;
    if (s->trace_cap > 0) {
        LaunchCtx c = ctx(s);
        if (launch_trace_rows(c, s->fwork, s->nfwork, s->trace_pos, s->trace, s->n_inst, s->trace_cap))
            return fail(PIC_EHIP, "trace launch");
    }
    return PIC_OK;
}

int enqueue_resort(pic_state *s)
{
    if (s->no_resort) return PIC_OK;
    LaunchCtx c = ctx(s);
    if (s->sched == PIC_SCHED_BATCHED) {
        if (launch_resort(c, s->cwork, s->ncwork, 0, s->n_inst, 1)) return fail(PIC_EHIP, "resort launch");
    } else {
        for (int i = 0; i < s->n_inst; i++)
            if (launch_resort(c, s->cwork + s->crange[i].off, s->crange[i].n, i, 1, i == s->n_inst - 1))
                return fail(PIC_EHIP, "resort launch");
    }
    return PIC_OK;
}

void drop_graphs(pic_state *s)
{
    for (int q = 0; q < 2; q++) {

        if (s->gexec_adj_fwd[q]) { (void)hipGraphExecDestroy(s->gexec_adj_fwd[q]); s->gexec_adj_fwd[q] = nullptr; }
    }
    if (s->gexec_adj_seg) { (void)hipGraphExecDestroy(s->gexec_adj_seg); s->gexec_adj_seg = nullptr; }
    for (int b = 0; b < 2; b++) {
        if (s->gexec_adj_rec[b]) { (void)hipGraphExecDestroy(s->gexec_adj_rec[b]); s->gexec_adj_rec[b] = nullptr; }
        if (s->gexec_adj_rev[b]) { (void)hipGraphExecDestroy(s->gexec_adj_rev[b]); s->gexec_adj_rev[b] = nullptr; }
    }
    for (auto &kv : s->gexec) (void)hipGraphExecDestroy(kv.second);
    s->gexec.clear();
}

// capture whatever `body` enqueues on the state's stream into an executable graph
// (the enqueue functions advance the host's parity as they record steps; a
// capture records without running, so the parity is put back afterwards)
template <class F> int capture_fn(pic_state *s, F body, hipGraphExec_t *out)
{
    hipGraph_t g = nullptr;
    const int par0 = s->parity;
    HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    int rc = body();
    s->parity = par0;
    hipError_t e = hipStreamEndCapture(s->stream, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(PIC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PIC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return PIC_OK;
}

int capture(pic_state *s, int k, bool with_resort, hipGraphExec_t *out)
{
    hipGraph_t g = nullptr;
    const int par0 = s->parity;
    HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    int rc = PIC_OK;
    for (int i = 0; i < k && rc == PIC_OK; i++) rc = enqueue_step(s);
    if (rc == PIC_OK && with_resort) rc = enqueue_resort(s);
    s->parity = par0;
    hipError_t e = hipStreamEndCapture(s->stream, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(PIC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PIC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return PIC_OK;
}

template <class R>
int copy_plane_out(pic_state *s, const void *src, size_t n, double *host, double scale, bool is_j)
{
    if (is_j && s->fp32) {
        std::vector<int> tmp(n);
        HIP_TRY(hipMemcpyAsync(tmp.data(), src, n * 4, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        for (size_t i = 0; i < n; i++) host[i] = (double)tmp[i] * scale;
        return PIC_OK;
    }
    if (is_j) {
        HIP_TRY(hipMemcpyAsync(host, src, n * 8, hipMemcpyDeviceToHost, s->stream));
        return hipStreamSynchronize(s->stream) == hipSuccess ? PIC_OK : fail(PIC_EHIP, "sync");
    }
    std::vector<R> tmp(n);
    HIP_TRY(hipMemcpyAsync(tmp.data(), src, n * sizeof(R), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (size_t i = 0; i < n; i++) host[i] = (double)tmp[i];
    return PIC_OK;
}

template <class R>
int copy_plane_in(pic_state *s, void *dst, size_t n, const double *host)
{
    std::vector<R> tmp(n);
    for (size_t i = 0; i < n; i++) tmp[i] = (R)host[i];
    HIP_TRY(hipMemcpyAsync(dst, tmp.data(), n * sizeof(R), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return PIC_OK;
}

template <class R>
int get_particles(pic_state *s, int inst, double *pos[3], double *mom[3])
{
    const InstDesc &D = s->desc[inst];
    const size_t n = (size_t)D.np;
    std::vector<int> idx(n), pid(n);
    std::vector<R> off[3], u[3];
    HIP_TRY(hipMemcpyAsync(idx.data(), D.pidx, n * 4, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(pid.data(), D.ppid, n * 4, hipMemcpyDeviceToHost, s->stream));
    for (int a = 0; a < 3; a++) {
        u[a].resize(n);
        HIP_TRY(hipMemcpyAsync(u[a].data(), D.pu[a], n * sizeof(R), hipMemcpyDeviceToHost, s->stream));
        if (D.poff[a]) {
            off[a].resize(n);
            HIP_TRY(hipMemcpyAsync(off[a].data(), D.poff[a], n * sizeof(R), hipMemcpyDeviceToHost, s->stream));
        }
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (size_t j = 0; j < n; j++) {
        const int i = pid[j];
        if (i < 0 || (size_t)i >= n) return fail(PIC_ESTATE, "corrupt particle ids");
        int c[3];
        if (s->dims == 2) unpack_cell<2>((unsigned)idx[j], c);
        else unpack_cell<3>((unsigned)idx[j], c);
        for (int a = 0; a < 3; a++) {
            if (mom[a]) mom[a][i] = (double)u[a][j];
            if (pos[a] && D.poff[a]) pos[a][i] = ((double)c[a] + (double)off[a][j]) * D.d[a];
        }
    }
    return PIC_OK;
}

}  // namespace

// ==================================================================== C ABI

extern "C" const char *pic_strerror(int code)
{
    switch (code) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument";
    case PIC_ECOURANT: return "time step violates the Yee Courant limit";
    case PIC_EPSI: return "correction polynomials not positive on [0,1] or singular interpolation";
    case PIC_ENOMEM: return "device arena too small";
    case PIC_EHIP: return "HIP runtime error";
    case PIC_ENONFINITE: return "non-finite value in fields or particles";
    case PIC_EPARTICLE: return "particle moved a full cell or more in one step";
    case PIC_EUNSUPPORTED: return "configuration not supported by this library";
    case PIC_ESTATE: return "invalid state";
    case PIC_ERANGE: return "current outside the fixed-point range of the float-mode current planes";
    }
    return "unknown error";
}

extern "C" const char *pic_last_error(void) { return g_last_error.c_str(); }

extern "C" int pic_plan(const pic_config *cfgs, int n_inst, const int64_t *n_particles, size_t *arena_bytes)
{
    if (!cfgs || n_inst < 1 || !n_particles || !arena_bytes) return fail(PIC_EINVAL, "null argument");
    for (int i = 0; i < n_inst; i++) {
        int rc = validate(cfgs[i], i);
        if (rc) return rc;
        if (cfgs[i].dims != cfgs[0].dims || cfgs[i].precision != cfgs[0].precision ||
            cfgs[i].shape_order != cfgs[0].shape_order || cfgs[i].adjoint_steps != cfgs[0].adjoint_steps ||
            cfgs[i].interp != cfgs[0].interp || cfgs[i].solver != cfgs[0].solver ||
            (cfgs[i].correction == PIC_CORR_RATIO) != (cfgs[0].correction == PIC_CORR_RATIO) ||
            (cfgs[0].adjoint_steps > 0 && cfgs[i].adjoint_ckpt != cfgs[0].adjoint_ckpt))
            return fail(PIC_EINVAL, "all instances must share dims, precision, shape_order, interp, solver, the exact-ratio choice and adjoint sizes");
        // the particle kernels address an instance's particle arrays with 32-bit
        // byte offsets (p * sizeof(element)), so n * max(sizeof(R), 4) must stay
        // below 2^32: 2^30 particles in FP32, 2^29 in FP64
        const int64_t nmax = (int64_t)(UINT32_MAX / (cfgs[0].precision == PIC_FP64 ? 8u : 4u));
        if (n_particles[i] < 0 || n_particles[i] > nmax)
            return fail(PIC_EINVAL, "particle count must be in [0, " + std::to_string(nmax) +
                                        "] (32-bit byte offsets into the particle arrays)");
    }
    const std::vector<pic_config> rc = resolve_tiles(cfgs, n_inst);
    *arena_bytes = layout(nullptr, rc.data(), n_inst, n_particles, nullptr);
    return PIC_OK;
}

extern "C" int pic_init(const pic_config *cfgs, int n_inst, const pic_particles *parts, void *d_arena,
                        size_t arena_bytes, void *hip_stream, pic_state **out)
{
    if (!out || !parts || !d_arena) return fail(PIC_EINVAL, "null argument");
    *out = nullptr;
    std::vector<int64_t> np(n_inst > 0 ? n_inst : 0);
    for (int i = 0; i < n_inst; i++) {
        np[i] = parts[i].n;
        if (parts[i].n > 0 && (!parts[i].pos[0] || !parts[i].pos[2] || !parts[i].mom[0] || !parts[i].mom[1] ||
                               !parts[i].mom[2] || (cfgs[i].dims == 3 && !parts[i].pos[1])))
            return fail(PIC_EINVAL, "null particle array");
    }
    size_t need = 0;
    int rc = pic_plan(cfgs, n_inst, np.data(), &need);
    if (rc) return rc;
    if (arena_bytes < need) return fail(PIC_ENOMEM, "arena smaller than pic_plan reported");
    const std::vector<pic_config> resolved = resolve_tiles(cfgs, n_inst);
    cfgs = resolved.data();
    if (((uintptr_t)d_arena & 255) != 0) return fail(PIC_EINVAL, "arena must be 256-byte aligned");

    pic_state *s = new pic_state();
    s->n_inst = n_inst;
    s->dims = cfgs[0].dims;
    s->order = cfgs[0].shape_order;
    s->fp32 = cfgs[0].precision == PIC_FP32;
    s->ck = cfgs[0].solver == PIC_CK;
    s->ratio = cfgs[0].correction == PIC_CORR_RATIO;
    s->gather = cfgs[0].interp == PIC_UNIFORM ? GATHER_UNIFORM
              : cfgs[0].interp == PIC_MOMENTUM ? GATHER_NODAL : GATHER_GALERKIN;
    s->cfg.assign(cfgs, cfgs + n_inst);
    s->np = np;
    s->desc.resize(n_inst);
    s->arena = (char *)d_arena;
    s->arena_bytes = arena_bytes;
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return fail(PIC_EHIP, "hipStreamCreateWithFlags");
        }
        s->own_stream = true;
    }
    auto bail = [&](int code) { pic_destroy(s); return code; };
    layout(s, cfgs, n_inst, np.data(), s->arena);
    {
        const hipError_t e = hipMemsetAsync(s->arena, 0, need - 256, s->stream);
        if (e != hipSuccess)
            return bail(fail(PIC_EHIP, std::string("arena clear (") + std::to_string(need - 256) + " bytes): " +
                                           hipGetErrorString(e)));
    }
    s->block = cfgs[0].block ? cfgs[0].block : default_block();
    // 2D FP32 field tiles: taller tiles (fewer halo rows per output row) pay once
    // the launches are bandwidth-bound, measured on a 64-instance batch of 3.9 M
    // cells (seen 74 -> 60 us, Yee 111 -> 109 us per step); a single 512 x 512
    // grid is latency-bound and keeps the shorter ones (the options override)
    if (s->dims == 2 && s->fp32) {
        long long cells = 0;
        for (int i = 0; i < n_inst; i++) cells += (long long)cfgs[i].nx * cfgs[i].nz;
        if (cells > 4LL * 512 * 512) { s->seen_tz = 32; s->yee_tz = 16; }
    }
    // largest LDS window over the instances
    int maxsm = 0;
    if (hipDeviceGetAttribute(&maxsm, hipDeviceAttributeMaxSharedMemoryPerBlock, 0) != hipSuccess) maxsm = 65536;
    {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            s->cus = v;
    }
    for (int i = 0; i < n_inst; i++) {
        fill_desc(s->desc[i], cfgs[i], parts[i]);
        int tile[3], slack;
        tile_shape(cfgs[i], tile, slack);
        for (int a = 0; a < 3; a++) {
            int w = (s->dims == 2 && a == 1) ? 1 : tile[a] + slack + s->order + 2;
            s->wmax[a] = std::max(s->wmax[a], w);
        }
    }
    {
        // particle state larger than the 256 MB last-level cache (with room for the
        // fields): stream it past the caches (see the particle kernel)
        const size_t R = s->fp32 ? 4 : 8;
        size_t bytes = 0;
        for (int i = 0; i < n_inst; i++)
            bytes += (size_t)np[i] * (4 + (s->dims == 2 ? 2 : 3) * R + 3 * R);
        const int nts = bytes > ((size_t)192 << 20) ? 1 : 0;
        for (int i = 0; i < n_inst; i++) s->desc[i].nts = nts;
    }
    if (s->seen_tz == 32) {
        // large FP32 batches: the seen pass streams 128-row segments where the
        // stencil widths allow (measured on a 64-instance batch of 3.9 M cells:
        // seen 59.0 -> 56.3 us per step)
        const LaunchCtx c0 = ctx(s);
        s->seen_tz = seen_tz_eff(128, s->fp32, c0.hz, c0.hx);
    }
    if (s->dims == 2) {
        // square windows of pitch 24 or 32 let the 2D kernel address LDS with immediates
        const int w = std::max(s->wmax[0], s->wmax[2]);
        const int pw = w <= 24 ? 24 : (w <= 32 ? 32 : w);
        const int wm2[3] = {pw, 1, pw};
        if (pw != w || s->wmax[0] != s->wmax[2])
            if (particle_smem_bytes(2, s->fp32, wm2) <= (size_t)maxsm) { s->wmax[0] = pw; s->wmax[2] = pw; }
    }
    if (s->dims == 3 && s->order == 3 && s->fp32) {
        // cubic 3D (default tile 8 x 2 x 4): pitches 15 x 9 x 11 let the kernel
        // address LDS with immediates; the odd row pitch spreads a wave's 64-bit
        // current adds over more LDS banks than 16 would (3.32 against 3.40 ms)
        const int wp[3] = {15, 9, 11};
        if (s->wmax[0] <= wp[0] && s->wmax[1] <= wp[1] && s->wmax[2] <= wp[2] &&
            particle_smem_bytes(3, s->fp32, wp) <= (size_t)maxsm)
            for (int a = 0; a < 3; a++) s->wmax[a] = wp[a];
    }
    while (particle_smem_bytes(s->dims, s->fp32, s->wmax) > (size_t)maxsm) {
        // shrink the slack until the window fits (tiles then re-sort more often)
        bool shrunk = false;
        for (int a = 0; a < 3; a++)
            if (!(s->dims == 2 && a == 1) && s->wmax[a] > s->order + 3) { s->wmax[a]--; shrunk = true; }
        if (!shrunk) return bail(fail(PIC_EINVAL, "tile window does not fit in LDS"));
    }
    {
        // allow the dynamic LDS size on every particle kernel instantiation
        (void)maxsm;
    }
    for (int i = 0; i < n_inst; i++) {
        s->desc[i].trace = s->trace;
        s->desc[i].any_resort = s->any_resort;
        s->desc[i].defer = s->defer;
    }
    if (cfgs[0].adjoint_steps > 0) {
        s->adj_steps = cfgs[0].adjoint_steps;
        s->adj_k = cfgs[0].adjoint_ckpt;
        for (int a = 0; a < 3; a++) s->adj_wmax[a] = s->wmax[a];
        while (adjoint_smem_bytes(s->dims, s->fp32, s->adj_wmax) > (size_t)maxsm) {
            bool shrunk = false;
            for (int a = 0; a < 3; a++)
                if (!(s->dims == 2 && a == 1) && s->adj_wmax[a] > s->order + 3) { s->adj_wmax[a]--; shrunk = true; }
            if (!shrunk) return bail(fail(PIC_EINVAL, "adjoint tile window does not fit in LDS"));
        }
        s->adj_slots = tape_slots(cfgs[0]);
        // one descriptor table per tape slot: E/B, particles and tile boxes of that slot
        std::vector<InstDesc> td((size_t)s->adj_slots * n_inst);
        for (int k = 0; k < s->adj_slots; k++)
            for (int i = 0; i < n_inst; i++) {
                InstDesc d = s->desc[i];
                const Snap &sn = s->tape[i][k];
                for (int c = 0; c < 3; c++) {
                    d.E[0][c] = d.E[1][c] = sn.E[c];
                    d.B[0][c] = d.B[1][c] = sn.B[c];
                    d.poff[c] = sn.poff[c];
                    d.pu[c] = sn.pu[c];
                }
                d.pidx = sn.pidx;
                d.tbox = sn.tbox;
                if (s->dims == 2)
                    for (int c = 0; c < 3; c++) { d.Et[c] = sn.Et[c]; d.Bt[c] = sn.Bt[c]; }
                td[(size_t)k * n_inst + i] = d;
            }
        // 2D: the recomputed step k runs on the live state but writes its seen
        // fields into slot k and records E1, B2 and its starting particles there
        std::vector<InstDesc> rd((size_t)s->adj_slots * n_inst);
        for (int k = 0; k < s->adj_slots && s->dims == 2; k++)
            for (int i = 0; i < n_inst; i++) {
                InstDesc d = s->desc[i];
                const Snap &sn = s->tape[i][k];
                for (int c = 0; c < 3; c++) {
                    d.Et[c] = sn.Et[c];
                    d.Bt[c] = sn.Bt[c];
                    d.rE[c] = sn.E[c];
                    d.rB[c] = sn.B[c];
                    d.roff[c] = sn.poff[c];
                    d.ru[c] = sn.pu[c];
                }
                d.rpidx = sn.pidx;
                d.rtbox = sn.tbox;
                rd[(size_t)k * n_inst + i] = d;
            }
        if (hipMemcpyAsync(s->d_tape_desc, td.data(), td.size() * sizeof(InstDesc), hipMemcpyHostToDevice,
                           s->stream) != hipSuccess ||
            hipMemcpyAsync(s->d_rec_desc, rd.data(), rd.size() * sizeof(InstDesc), hipMemcpyHostToDevice,
                           s->stream) != hipSuccess ||
            hipStreamSynchronize(s->stream) != hipSuccess)
            return bail(fail(PIC_EHIP, "tape descriptor upload"));
    }
    if (hipMemcpyAsync(s->d_desc, s->desc.data(), n_inst * sizeof(InstDesc), hipMemcpyHostToDevice, s->stream) !=
        hipSuccess)
        return bail(fail(PIC_EHIP, "descriptor upload"));
    if ((rc = build_worklists(s))) return bail(rc);
    for (int i = 0; i < n_inst; i++) {
        rc = s->fp32 ? upload_particles<float>(s, i, parts[i]) : upload_particles<double>(s, i, parts[i]);
        if (rc) return bail(rc);
    }
    LaunchCtx c = ctx(s);
    if (launch_fill_bbox(c, 0, n_inst)) return bail(fail(PIC_EHIP, "bbox init"));
    if (launch_rho(c, s->pwork, s->npwork, s->fwork, s->nfwork, s->wmax, 1)) return bail(fail(PIC_EHIP, "rho0"));
    if (hipStreamSynchronize(s->stream) != hipSuccess) return bail(fail(PIC_EHIP, "init sync"));
    *out = s;
    return PIC_OK;
}

// ------------------------------------------------------------ static arena
// For callers that cannot allocate: the arena lives in a fixed device array.
// On the host, `scratch` names the symbol only, never device memory; its device
// address comes from hipGetSymbolAddress, once per device with that device
// current, and only that address is handed on.  One live state per device owns
// the array; pic_destroy releases it.
static __device__ __align__(256) unsigned char scratch[PIC_STATIC_ARENA_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices];             // device address of scratch, per device
const pic_state *g_static_owner[kMaxDevices];  // live state in that device's array
}  // namespace

extern "C" int pic_init_static(const pic_config *cfgs, int n_inst, const pic_particles *parts, void *hip_stream,
                               pic_state **out)
{
    if (!out || !parts || !cfgs) return fail(PIC_EINVAL, "null argument");
    *out = nullptr;
    if (!hip_stream) return fail(PIC_EINVAL, "pic_init_static: a stream is required (none is created)");
    if (n_inst < 1) return fail(PIC_EINVAL, "n_inst");
    std::vector<int64_t> np(n_inst);
    for (int i = 0; i < n_inst; i++) np[i] = parts[i].n;
    size_t need = 0;
    int rc = pic_plan(cfgs, n_inst, np.data(), &need);
    if (rc) return rc;
    if (need > (size_t)PIC_STATIC_ARENA_BYTES)
        return fail(PIC_ENOMEM, "pic_init_static: the instances need " + std::to_string(need) +
                                    " arena bytes; the static arena holds " +
                                    std::to_string((size_t)PIC_STATIC_ARENA_BYTES));
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(PIC_EHIP, "pic_init_static: current device");
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_owner[dev])
        return fail(PIC_ESTATE, "pic_init_static: the static arena of this device holds a live state");
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PIC_EHIP, std::string("pic_init_static: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_static_ptr[dev] = p;
    }
    rc = pic_init(cfgs, n_inst, parts, g_static_ptr[dev], (size_t)PIC_STATIC_ARENA_BYTES, hip_stream, out);
    if (rc) return rc;
    (*out)->static_dev = dev;
    g_static_owner[dev] = *out;
    return PIC_OK;
}

extern "C" int pic_set_schedule(pic_state *s, int sched, int use_graph)
{
    if (!s || (sched != PIC_SCHED_BATCHED && sched != PIC_SCHED_PLAIN)) return fail(PIC_EINVAL, "schedule");
    if (s->sched != sched || s->use_graph != (use_graph ? 1 : 0)) drop_graphs(s);
    s->sched = sched;
    s->use_graph = use_graph ? 1 : 0;
    return PIC_OK;
}

extern "C" int pic_set_option(pic_state *s, const char *name, int value)
{
    if (!s || !name) return fail(PIC_EINVAL, "pic_set_option");
    const std::string n(name);
    if (n == "yee_tile_z") {
        if (value != 4 && value != 8 && value != 16) return fail(PIC_EINVAL, "yee_tile_z must be 4, 8 or 16");
        s->yee_tz = yee_tz_eff(value, s->fp32);
    } else if (n == "seen_tile_z") {
        if (value != 8 && value != 16 && value != 32 && value != 64 && value != 128)
            return fail(PIC_EINVAL, "seen_tile_z must be 8, 16, 32, 64 or 128");
        const LaunchCtx c = ctx(s);
        s->seen_tz = seen_tz_eff(value, s->fp32, c.hz, c.hx);
    } else if (n == "resort_every") {
        if (value < 1 || value > 1024) return fail(PIC_EINVAL, "resort_every must be in [1, 1024]");
        s->graph_k = value;
    } else if (n == "particle_block") {
        if (value != 256 && value != 512) return fail(PIC_EINVAL, "particle_block must be 256 or 512");
        s->block = value;
    } else if (n == "particle_waves4") {
        if (value != 0 && value != 1) return fail(PIC_EINVAL, "particle_waves4 must be 0 or 1");
        s->waves4 = value;
    } else if (n == "particle_prefetch") {
        if (value != 0 && value != 1) return fail(PIC_EINVAL, "particle_prefetch must be 0 or 1");
        s->prefetch = value;
    } else if (n == "particle_defer") {
        if (value < -1 || value > 1) return fail(PIC_EINVAL, "particle_defer must be -1, 0 or 1");
        s->defer_mode = value;
    } else if (n == "current_quantum_shift") {
        if (!s->fp32 || value < 0 || value > 24 || s->step != 0)
            return fail(PIC_EINVAL, "current_quantum_shift: float mode, in [0, 24], before the first step");
        for (InstDesc &d : s->desc) { d.jshift = value; d.jqg = d.jq * std::ldexp(1.0, value); }
        HIP_TRY(hipMemcpyAsync(s->d_desc, s->desc.data(), s->n_inst * sizeof(InstDesc), hipMemcpyHostToDevice,
                               s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    } else {
        return fail(PIC_EINVAL, "unknown option " + n);
    }
    drop_graphs(s);
    return build_worklists(s);
}

extern "C" int pic_get_option(pic_state *s, const char *name, int *value)
{
    if (!s || !name || !value) return fail(PIC_EINVAL, "pic_get_option");
    const std::string n(name);
    if (n == "yee_tile_z") *value = s->yee_tz;
    else if (n == "seen_tile_z") *value = s->seen_tz;
    else if (n == "resort_every") *value = s->graph_k;
    else if (n == "particle_block") *value = s->block;
    else if (n == "particle_waves4") *value = s->waves4;
    else if (n == "particle_prefetch") *value = s->prefetch;
    else if (n == "particle_defer") *value = s->defer_mode;
    else if (n == "current_quantum_shift") *value = s->desc.empty() ? 0 : s->desc[0].jshift;
    else return fail(PIC_EINVAL, "unknown option " + n);
    return PIC_OK;
}

namespace {

// The pieces a graph-replayed run of nsteps from the current state is made
// of: steps up to the next multiple of the re-sort period (with the re-sort
// check at its end when it gets there), whole periods (each ending with the
// check), and the remaining steps.  Eager stepping checks at the same steps;
// no check while re-sorting is suspended (between the adjoint calls).
struct Piece { int len, resort; };
std::vector<Piece> plan_run(const pic_state *s, int nsteps)
{
    std::vector<Piece> out;
    long long step = s->step;
    int n = 0;
    while (n < nsteps) {
        const int to_check = s->graph_k - (int)(step % s->graph_k);
        const int len = std::min(to_check, nsteps - n);
        out.push_back(Piece{len, (len == to_check && !s->no_resort) ? 1 : 0});
        step += len;
        n += len;
    }
    return out;
}

// the graph of one piece starting from parity q, captured on first use
int piece_graph(pic_state *s, const Piece &p, int q, hipGraphExec_t *out)
{
    const auto key = std::make_tuple(p.len, p.resort, q);
    auto it = s->gexec.find(key);
    if (it != s->gexec.end()) { *out = it->second; return PIC_OK; }
    const int par0 = s->parity;
    s->parity = q;
    hipGraphExec_t g = nullptr;
    const int rc = capture(s, p.len, p.resort != 0, &g);
    s->parity = par0;
    if (rc) return rc;
    s->gexec[key] = g;
    *out = g;
    return PIC_OK;
}

}  // namespace

extern "C" int pic_step(pic_state *s, int nsteps)
{
    if (!s || nsteps < 0) return fail(PIC_EINVAL, "pic_step");
    int rc;
    if (!s->use_graph) {
        for (int n = 0; n < nsteps; n++) {
            if ((rc = enqueue_step(s))) return rc;
            s->step++;
            if (s->step % s->graph_k == 0 && (rc = enqueue_resort(s))) return rc;
        }
        return PIC_OK;
    }
    for (const Piece &p : plan_run(s, nsteps)) {
        hipGraphExec_t g = nullptr;
        if ((rc = piece_graph(s, p, s->parity, &g))) return rc;
        HIP_TRY(hipGraphLaunch(g, s->stream));
        s->parity ^= p.len & 1;
        s->step += p.len;
    }
    return PIC_OK;
}

extern "C" int pic_prepare(pic_state *s, int nsteps)
{
    if (!s || nsteps < 0) return fail(PIC_EINVAL, "pic_prepare");
    if (!s->use_graph) return PIC_OK;
    int q = s->parity;
    for (const Piece &p : plan_run(s, nsteps)) {
        hipGraphExec_t g = nullptr;
        const int rc = piece_graph(s, p, q, &g);
        if (rc) return rc;
        q ^= p.len & 1;
    }
    return PIC_OK;
}

extern "C" int pic_fields(pic_state *s, int inst, int which, int comp, double *host, size_t n, int dir)
{
    if (!s || inst < 0 || inst >= s->n_inst || comp < 0 || comp > 2 || !host) return fail(PIC_EINVAL, "pic_fields");
    const InstDesc &D = s->desc[inst];
    if (n != (size_t)D.ncell) return fail(PIC_EINVAL, "pic_fields: n must equal nx*ny*nz");
    void *src = nullptr;
    bool is_j = false, is_rho = false;
    switch (which) {
    case PIC_FIELD_E: src = D.E[s->parity][comp]; break;
    case PIC_FIELD_B: src = D.B[s->parity][comp]; break;
    case PIC_FIELD_J: src = D.J[s->parity][comp]; is_j = true; break;
    case PIC_FIELD_SEEN_E: src = D.Et[comp]; break;
    case PIC_FIELD_SEEN_B: src = D.Bt[comp]; break;
    case PIC_FIELD_RHO: is_rho = true; break;
    default: return fail(PIC_EINVAL, "pic_fields: which");
    }
    if (dir == PIC_SET) {
        if (which != PIC_FIELD_E && which != PIC_FIELD_B) return fail(PIC_EINVAL, "SET allowed for E and B only");
        return s->fp32 ? copy_plane_in<float>(s, src, n, host) : copy_plane_in<double>(s, src, n, host);
    }
    if (dir != PIC_GET) return fail(PIC_EINVAL, "pic_fields: dir");
    if (is_rho) {
        LaunchCtx c = ctx(s);
        const Range &pr = s->prange[inst], &fr = s->frange[inst];
        if (launch_rho(c, s->pwork + pr.off, pr.n, s->fwork + fr.off, fr.n, s->wmax, 0)) return fail(PIC_EHIP, "rho");
        HIP_TRY(hipMemcpyAsync(host, D.rho, n * 8, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        return PIC_OK;
    }
    return s->fp32 ? copy_plane_out<float>(s, src, n, host, D.jqg, is_j)
                   : copy_plane_out<double>(s, src, n, host, D.jqg, is_j);
}

extern "C" int pic_get_particles(pic_state *s, int inst, double *pos[3], double *mom[3], int64_t n)
{
    if (!s || inst < 0 || inst >= s->n_inst || !pos || !mom) return fail(PIC_EINVAL, "pic_get_particles");
    if (n != s->desc[inst].np) return fail(PIC_EINVAL, "pic_get_particles: n mismatch");
    return s->fp32 ? get_particles<float>(s, inst, pos, mom) : get_particles<double>(s, inst, pos, mom);
}

extern "C" int pic_diag(pic_state *s, int inst, pic_diag_t *out)
{
    if (!s || inst < 0 || inst >= s->n_inst || !out) return fail(PIC_EINVAL, "pic_diag");
    const InstDesc &D = s->desc[inst];
    LaunchCtx c = ctx(s);
    const Range &pr = s->prange[inst], &fr = s->frange[inst];
    if (launch_diag(c, s->fwork + fr.off, fr.n, s->pwork + pr.off, pr.n, s->wmax)) return fail(PIC_EHIP, "diag");
    double dg[DG_COUNT];
    int fl[FLAG_COUNT];
    HIP_TRY(hipMemcpyAsync(dg, D.diag, sizeof dg, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(fl, D.flags, sizeof fl, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::memset(out, 0, sizeof *out);
    for (int k = 0; k < 3; k++) { out->WE[k] = dg[DG_WE + k]; out->WB[k] = dg[DG_WB + k]; }
    out->Wkin = dg[DG_WKIN];
    out->gauss_l2 = std::sqrt(dg[DG_G2]);
    out->gauss_linf = dg[DG_GMAX];
    out->charge = dg[DG_CHARGE];
    out->rho_max = dg[DG_RHOMAX];
    out->n_particles = D.np;
    out->step = s->step;
    out->nonfinite = dg[DG_NONFIN] > 0 ? 1 : 0;
    for (int k = 0; k < 6; k++) {
        double v = k < 3 ? out->WE[k] : out->WB[k - 3];
        if (!std::isfinite(v)) out->nonfinite = 1;
    }
    out->particle_error = fl[FLAG_PERR] ? 1 : 0;
    out->resorts = fl[FLAG_NRESORT];
    out->slow_tiles = fl[FLAG_SLOW];
    out->current_range = fl[FLAG_JRANGE] ? 1 : 0;
    if (out->nonfinite) return fail(PIC_ENONFINITE, "non-finite value found");
    if (out->particle_error) return fail(PIC_EPARTICLE, "particle moved a full cell");
    if (out->current_range) return fail(PIC_ERANGE, "current outside the 32-bit fixed-point range");
    return PIC_OK;
}

extern "C" int pic_read_trace(pic_state *s, int inst, double *host_out, int max_rows, int *count)
{
    if (!s || inst < 0 || inst >= s->n_inst || !host_out || !count) return fail(PIC_EINVAL, "pic_read_trace");
    *count = 0;
    if (s->trace_cap <= 0) return PIC_OK;
    int pos = 0;
    HIP_TRY(hipMemcpyAsync(&pos, s->trace_pos, sizeof pos, hipMemcpyDeviceToHost, s->stream));
    std::vector<double> all((size_t)s->trace_cap * s->n_inst * 6);
    HIP_TRY(hipMemcpyAsync(all.data(), s->trace, all.size() * 8, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const int rows = std::min(std::min(pos, s->trace_cap - 1), max_rows);
    const int first = pos - rows;
    for (int r = 0; r < rows; r++) {
        const int slot = (first + r) % s->trace_cap;
        for (int k = 0; k < 6; k++) host_out[r * 6 + k] = all[((size_t)slot * s->n_inst + inst) * 6 + k];
    }
    *count = rows;
    return PIC_OK;
}

extern "C" int pic_profile(pic_state *s, int nsteps, pic_timing_t *out)
{
    if (!s || !out || nsteps < 1) return fail(PIC_EINVAL, "pic_profile");
    std::memset(out, 0, sizeof *out);
    hipEvent_t ev[5];
    for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    double acc[4] = {0, 0, 0, 0}, total = 0;
    int nres = 0;
    LaunchCtx c = ctx(s);
    for (int n = 0; n < nsteps; n++) {
        const Range f{0, s->nfwork}, p{0, s->npwork};
        HIP_TRY(hipEventRecord(ev[0], s->stream));
        c.par = s->parity;
        if (launch_yee(c, s->fwork, f.n, s->ywork, s->nywork)) return fail(PIC_EHIP, "yee");
        c.par ^= 1;
        s->parity ^= 1;
        HIP_TRY(hipEventRecord(ev[1], s->stream));
        if (launch_seen(c, s->fwork, f.n, s->swork, s->nswork)) return fail(PIC_EHIP, "seen");
        HIP_TRY(hipEventRecord(ev[2], s->stream));
        if (launch_particles(c, s->pwork, p.n, 0, s->block, s->wmax)) return fail(PIC_EHIP, "particles");
        HIP_TRY(hipEventRecord(ev[3], s->stream));
        s->step++;
        const bool res = s->step % s->graph_k == 0;
        if (res && launch_resort(c, s->cwork, s->ncwork, 0, s->n_inst, 1)) return fail(PIC_EHIP, "resort");
        HIP_TRY(hipEventRecord(ev[4], s->stream));
        HIP_TRY(hipEventSynchronize(ev[4]));
        float t[4];
        for (int k = 0; k < 4; k++) HIP_TRY(hipEventElapsedTime(&t[k], ev[k], ev[k + 1]));
        for (int k = 0; k < 4; k++) acc[k] += t[k];
        total += t[0] + t[1] + t[2] + t[3];
        nres += res;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    out->yee_ms = acc[0] / nsteps;
    out->seen_ms = acc[1] / nsteps;
    out->particle_ms = acc[2] / nsteps;
    out->resort_ms = nres ? acc[3] / nres : 0.0;
    out->step_ms = total / nsteps;
    out->steps = nsteps;
    return PIC_OK;
}

namespace {

// save: from the current set of E, B, J planes; restore: into set 0 (the caller
// makes set 0 current once every instance is restored)
// E, B (and J) of set q, the particles and the tile boxes of one instance to
// (save) or from a snapshot, in one copy launch
int snap_copy(pic_state *s, int inst, const Snap &sn, bool save, bool with_j)
{
    const InstDesc &D = s->desc[inst];
    const size_t R = s->fp32 ? 4 : 8;
    const int q = save ? s->parity : 0;
    CopyList L;
    bool aligned = true;
    auto add = [&](void *live, void *snapp, size_t bytes) {
        if (!bytes || !live || !snapp) return;
        L.src[L.n] = save ? live : snapp;
        L.dst[L.n] = save ? snapp : live;
        L.bytes[L.n] = (long long)bytes;
        aligned = aligned && ((uintptr_t)live % 16 == 0) && ((uintptr_t)snapp % 16 == 0) && bytes % 4 == 0;
        L.n++;
    };
    add(D.E[q][0], sn.E[0], region_fields(D, R));
    if (with_j) add(D.J[q][0], sn.J[0], region_j(D, s->fp32 ? 4 : 8));
    if (D.np > 0) add(D.pidx, sn.pidx, region_particles(D, R));
    add(D.tbox, sn.tbox, (size_t)D.ntiles * 6 * 4);
    if (aligned) {
        if (launch_copy_list(s->stream, L)) return fail(PIC_EHIP, "snapshot copy");
        return PIC_OK;
    }
    for (int k = 0; k < L.n; k++)
        HIP_TRY(hipMemcpyAsync(L.dst[k], L.src[k], (size_t)L.bytes[k], hipMemcpyDeviceToDevice, s->stream));
    return PIC_OK;
}

}  // namespace

namespace {

int gradient_preconditions(pic_state *s)
{
    if (s->adj_steps <= 0) return fail(PIC_ESTATE, "gradient runs were not planned (adjoint_steps = 0)");
    for (int i = 0; i < s->n_inst; i++)
        if (!s->cfg[i].correction) return fail(PIC_EINVAL, "gradient needs the correction enabled");
    return PIC_OK;
}

int forward_step_eager(pic_state *s)
{
    LaunchCtx live = ctx(s);
    if (launch_yee(live, s->fwork, s->nfwork, s->ywork, s->nywork)) return fail(PIC_EHIP, "yee");
    live.par ^= 1;
    if (launch_seen(live, s->fwork, s->nfwork, s->swork, s->nswork)) return fail(PIC_EHIP, "seen");
    if (launch_particles(live, s->pwork, s->npwork, 0, s->block, s->wmax)) return fail(PIC_EHIP, "particles");
    s->parity ^= 1;
    return PIC_OK;
}

// recompute m steps from the restored checkpoint while recording the tape
// slots slot0 .. slot0 + m - 1 (main stream)
int enqueue_recompute(pic_state *s, int m, int slot0)
{
    LaunchCtx live = ctx(s);
    int rc = PIC_OK;
    for (int k = 0; k < m && rc == PIC_OK; k++) {
        const int slot = slot0 + k;
        if (s->dims == 2) {
            // the kernels write the tape themselves (record descriptors)
            LaunchCtx rec = live;
            rec.desc = s->d_rec_desc + (size_t)slot * s->n_inst;
            rec.record = 1;
            rec.par = s->parity;
            if (launch_yee(rec, s->fwork, s->nfwork, s->ywork, s->nywork)) return fail(PIC_EHIP, "recompute");
            rec.par ^= 1;
            if (launch_seen(rec, s->fwork, s->nfwork, s->swork, s->nswork) ||
                launch_particles(rec, s->pwork, s->npwork, 0, s->block, s->wmax))
                return fail(PIC_EHIP, "recompute");
            s->parity ^= 1;
            continue;
        }
        for (int i = 0; i < s->n_inst && rc == PIC_OK; i++) rc = snap_copy_particles(s, i, s->tape[i][slot], true);
        if (rc) break;
        LaunchCtx c = live;
        c.par = s->parity;
        if (launch_yee(c, s->fwork, s->nfwork, s->ywork, s->nywork)) return fail(PIC_EHIP, "recompute");
        c.par ^= 1;
        if (launch_seen(c, s->fwork, s->nfwork, s->swork, s->nswork)) return fail(PIC_EHIP, "recompute");
        for (int i = 0; i < s->n_inst && rc == PIC_OK; i++) rc = snap_copy_fields(s, i, s->tape[i][slot], c.par);
        if (rc) break;
        if (launch_particles(c, s->pwork, s->npwork, 0, s->block, s->wmax)) return fail(PIC_EHIP, "recompute");
        s->parity ^= 1;
    }
    return rc;
}

// reverse the m steps recorded in slots slot0 .. slot0 + m - 1, last first, on
// `stream`.  The reverse kernels read the tape and the adjoint planes only,
// never the live E, B, J or particles (in 3D they recompute the seen fields
// into the live planes, so 3D runs them serially after the recompute).
int enqueue_reverse(pic_state *s, int m, int slot0, hipStream_t stream)
{
    LaunchCtx live = ctx(s);
    live.stream = stream;
    for (int k = m - 1; k >= 0; k--) {
        LaunchCtx tp = live;
        tp.desc = s->d_tape_desc + (size_t)(slot0 + k) * s->n_inst;
        if (launch_adj_step(live, tp, s->fwork, s->nfwork, s->swork, s->nswork, s->awork, s->nawork, s->pwork,
                            s->npwork, 256, s->adj_wmax))
            return fail(PIC_EHIP, "adjoint step");
    }
    return PIC_OK;
}

// one segment, serially on the main stream: recompute, then reverse
int enqueue_segment(pic_state *s, int m)
{
    const int rc = enqueue_recompute(s, m, 0);
    return rc ? rc : enqueue_reverse(s, m, 0, s->stream);
}

int enqueue_forward_steps(pic_state *s, int m)
{
    for (int n = 0; n < m; n++) {
        int rc = forward_step_eager(s);
        if (rc) return rc;
    }
    return PIC_OK;
}

}  // namespace

extern "C" int pic_adjoint_forward(pic_state *s, int nsteps, double *loss)
{
    if (!s || !loss || nsteps < 1) return fail(PIC_EINVAL, "pic_adjoint_forward");
    int rc = gradient_preconditions(s);
    if (rc) return rc;
    if (nsteps > s->adj_steps) return fail(PIC_EINVAL, "nsteps exceeds the planned adjoint_steps");
    const int K = s->adj_k, nseg = (nsteps + K - 1) / K;
    s->no_resort = true;      // particle order must stay fixed until the backward sweep
    s->adj_pending = 0;
    for (int seg = 0; seg < nseg && rc == PIC_OK; seg++) {
        for (int i = 0; i < s->n_inst && rc == PIC_OK; i++) rc = snap_copy(s, i, s->ckpt[i][seg], true, true);
        if (rc) break;
        const int m = std::min(K, nsteps - seg * K);
        if (m == K && s->use_graph) {
            const int q = s->parity;
            if (!s->gexec_adj_fwd[q] &&
                (rc = capture_fn(s, [&]() { return enqueue_forward_steps(s, K); }, &s->gexec_adj_fwd[q])))
                break;
            if (hipGraphLaunch(s->gexec_adj_fwd[q], s->stream) != hipSuccess) rc = fail(PIC_EHIP, "graph launch");
            s->parity ^= K & 1;
        } else {
            rc = enqueue_forward_steps(s, m);
        }
    }
    for (int i = 0; i < s->n_inst && rc == PIC_OK; i++) rc = snap_copy(s, i, s->ckpt[i][nseg], true, true);
    if (rc) { s->no_resort = false; return rc; }
    s->step += nsteps;
    // W of the final fields (the seed kernel also writes lambda_E, lambda_B, lambda_J)
    for (int i = 0; i < s->n_inst; i++)
        HIP_TRY(hipMemsetAsync(s->desc[i].grad, 0, 16 * PIC_GRAD_COPIES * sizeof(double), s->stream));
    LaunchCtx live = ctx(s);
    if (launch_adj_seed(live, s->fwork, s->nfwork, s->cwork, s->ncwork)) return fail(PIC_EHIP, "seed");
    std::vector<double> g(16);
    for (int i = 0; i < s->n_inst; i++) {
        HIP_TRY(hipMemcpyAsync(g.data(), s->desc[i].grad, 16 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        loss[i] = g[9];
    }
    s->adj_pending = nsteps;
    return PIC_OK;
}

namespace {

// the reverse stream and its events, made by the first 2D reverse sweep (so
// that pic_init itself creates none)
int ensure_rstream(pic_state *s)
{
    if (s->rstream) return PIC_OK;
    if (hipStreamCreateWithFlags(&s->rstream, hipStreamNonBlocking) != hipSuccess) {
        s->rstream = nullptr;
        return fail(PIC_EHIP, "reverse stream");
    }
    for (int b = 0; b < 2; b++) {
        HIP_TRY(hipEventCreateWithFlags(&s->ev_rec[b], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&s->ev_rev[b], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
    return PIC_OK;
}

// 2D reverse sweep in two streams.  Segment j (the last segment first) is
// recomputed on the main stream into tape bank j % 2 while segment j - 1 is
// reversed on rstream from the other bank.  A bank is refilled only after the
// reverse that read it has finished (ev_rev), a reverse starts after its
// recompute (ev_rec), and the reverses run in order on one stream, so the
// adjoint state passes from one segment to the next as in the serial sweep.
int backward_pipelined(pic_state *s, int nsteps)
{
    const int K = s->adj_k, nseg = (nsteps + K - 1) / K;
    int rc = ensure_rstream(s);
    if (rc) return rc;
    // the reverse stream starts after the work already on the main stream (the seed)
    HIP_TRY(hipEventRecord(s->ev_join, s->stream));
    HIP_TRY(hipStreamWaitEvent(s->rstream, s->ev_join, 0));
    for (int j = 0; j < nseg && rc == PIC_OK; j++) {
        const int seg = nseg - 1 - j, b = j & 1, slot0 = b * K;
        const int m = std::min(K, nsteps - seg * K);
        if (j >= 2) HIP_TRY(hipStreamWaitEvent(s->stream, s->ev_rev[b], 0));
        for (int i = 0; i < s->n_inst && rc == PIC_OK; i++) rc = snap_copy(s, i, s->ckpt[i][seg], false, true);
        if (rc) break;
        s->parity = 0;
        if (m == K && s->use_graph) {
            if (!s->gexec_adj_rec[b] &&
                (rc = capture_fn(s, [&]() { return enqueue_recompute(s, K, slot0); }, &s->gexec_adj_rec[b])))
                break;
            if (hipGraphLaunch(s->gexec_adj_rec[b], s->stream) != hipSuccess) { rc = fail(PIC_EHIP, "graph launch"); break; }
        } else if ((rc = enqueue_recompute(s, m, slot0))) {
            break;
        }
        HIP_TRY(hipEventRecord(s->ev_rec[b], s->stream));
        HIP_TRY(hipStreamWaitEvent(s->rstream, s->ev_rec[b], 0));
        if (m == K && s->use_graph) {
            // captured on the main stream, replayed on the reverse one
            if (!s->gexec_adj_rev[b] &&
                (rc = capture_fn(s, [&]() { return enqueue_reverse(s, K, slot0, s->stream); }, &s->gexec_adj_rev[b])))
                break;
            if (hipGraphLaunch(s->gexec_adj_rev[b], s->rstream) != hipSuccess) { rc = fail(PIC_EHIP, "graph launch"); break; }
        } else if ((rc = enqueue_reverse(s, m, slot0, s->rstream))) {
            break;
        }
        HIP_TRY(hipEventRecord(s->ev_rev[b], s->rstream));
    }
    // the main stream goes on after the last reverse
    HIP_TRY(hipEventRecord(s->ev_join, s->rstream));
    HIP_TRY(hipStreamWaitEvent(s->stream, s->ev_join, 0));
    return rc;
}

}  // namespace

extern "C" int pic_adjoint_backward(pic_state *s, double *grad)
{
    if (!s || !grad) return fail(PIC_EINVAL, "pic_adjoint_backward");
    const int nsteps = s->adj_pending;
    if (nsteps <= 0) return fail(PIC_ESTATE, "pic_adjoint_forward must run first");
    const int K = s->adj_k, nseg = (nsteps + K - 1) / K;
    int rc = PIC_OK;
    if (s->dims == 2) {
        rc = backward_pipelined(s, nsteps);
    } else {
        for (int seg = nseg - 1; seg >= 0 && rc == PIC_OK; seg--) {
            for (int i = 0; i < s->n_inst && rc == PIC_OK; i++) rc = snap_copy(s, i, s->ckpt[i][seg], false, true);
            if (rc) break;
            s->parity = 0;
            const int m = std::min(K, nsteps - seg * K);
            if (m == K && s->use_graph) {
                if (!s->gexec_adj_seg &&
                    (rc = capture_fn(s, [&]() { return enqueue_segment(s, K); }, &s->gexec_adj_seg)))
                    break;
                if (hipGraphLaunch(s->gexec_adj_seg, s->stream) != hipSuccess) rc = fail(PIC_EHIP, "graph launch");
            } else {
                rc = enqueue_segment(s, m);
            }
        }
    }
    // back to the forward end state
    for (int i = 0; i < s->n_inst && rc == PIC_OK; i++) rc = snap_copy(s, i, s->ckpt[i][nseg], false, true);
    s->parity = 0;
    s->no_resort = false;
    s->adj_pending = 0;
    if (rc) return rc;
    std::vector<double> g(16 * PIC_GRAD_COPIES);
    for (int i = 0; i < s->n_inst; i++) {
        HIP_TRY(hipMemcpyAsync(g.data(), s->desc[i].grad, g.size() * sizeof(double), hipMemcpyDeviceToHost,
                               s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        for (int j = 0; j < 9; j++) {
            double v = 0.0;
            for (int k = 0; k < PIC_GRAD_COPIES; k++) v += g[16 * k + j];
            grad[i * 9 + j] = j <= s->desc[i].psi_deg ? v : 0.0;
        }
    }
    return PIC_OK;
}

extern "C" int pic_info(pic_state *s, int *n_inst, int64_t *n_particles, int64_t *n_cells)
{
    if (!s) return fail(PIC_EINVAL, "pic_info");
    int64_t np = 0, nc = 0;
    for (int i = 0; i < s->n_inst; i++) { np += s->desc[i].np; nc += s->desc[i].ncell; }
    if (n_inst) *n_inst = s->n_inst;
    if (n_particles) *n_particles = np;
    if (n_cells) *n_cells = nc;
    return PIC_OK;
}

extern "C" void pic_destroy(pic_state *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->rstream) (void)hipStreamSynchronize(s->rstream);
    drop_graphs(s);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    if (s->rstream) (void)hipStreamDestroy(s->rstream);
    for (int b = 0; b < 2; b++) {
        if (s->ev_rec[b]) (void)hipEventDestroy(s->ev_rec[b]);
        if (s->ev_rev[b]) (void)hipEventDestroy(s->ev_rev[b]);
    }
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    if (s->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static_owner[s->static_dev] == s) g_static_owner[s->static_dev] = nullptr;
    }
    delete s;
}
