// C ABI of the Teukolsky m-mode stepper: context management, workspace
// layout on caller-owned device memory, stepping (eager or HIP graphs),
// field I/O and waveform extraction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tk_internal.h"
#include "tk_kernels.h"
#include "tk_layer_launch.h"
#include "tk_scratch.h"

using namespace tk;

struct tk_ctx {
    std::vector<HostInst> inst;
    tk_precision prec = TK_FP64;
    hipStream_t stream = nullptr;
    std::string err;
    int device = 0;
    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0, need = 0;
    size_t off_ctl = 0, off_inst = 0, off_blocks = 0, off_work = 0;
    std::vector<int2> blocks;          // two-pass decomposition
    std::vector<WorkItem> work;        // fused decomposition
    int work_rows = 0;                 // rows_per_tile the work list was built for
    int work_cols = 0;                 // strip width it was built for
    bool work_chunked = false;         // it holds chunks of rows (the two-step pass takes its chunked form)
    size_t work_cap = 0;               // capacity of the work list area (items)
    std::vector<DevInst> hdev;         // host mirror of the device descriptors
    std::vector<std::vector<Radial>> hrad;   // host copies of the coefficient tables
    std::vector<std::vector<Angular>> hang;
    std::vector<std::vector<AngularF>> hangf;
    // hyperboloidal layer: any instance with one makes the context step with
    // the marching kernels' layered form, or the layer's two passes (FP64,
    // TWO_PASS)
    bool layered = false;
    size_t off_linst = 0;              // LayerInst per instance
    std::vector<size_t> off_lay;       // LayerTab table per instance (layered ones)
    size_t off_lwork = 0, lwork_cap = 0;  // the layer kernels' work list area (items)
    std::vector<WorkItem> lwork;
    int lwork_rows = -1;               // rows per chunk it was built for
    long long step = 0;
    int cur = 0;  // state buffer holding u^step (mirror of the device control block)
    tk_tuning tuning{TK_KERNEL_AUTO, 0, 0, 3, TK_TUNE_NT_STORES, 0};
    // captured graph (steps, kernel, rows) for replay
    hipGraphExec_t gexec = nullptr;
    int g_steps = 0, g_flips = 0, g_kernel = -1, g_rows = -1, g_pf = -1, g_flags = -1, g_waves = -1;
    tk_counters counters{0, 0, 0};
    // the autotuner's timing events, created with the workspace binding
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

thread_local std::string g_err;

tk_status fail(tk_ctx *c, tk_status s, const std::string &msg)
{
    if (c)
        c->err = msg;
    else
        g_err = msg;
    return s;
}

#define TK_HIP(ctx, call)                                                                                  \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return fail((ctx), TK_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));            \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

std::string validate(const tk_instance_desc &d)
{
    char b[256];
    if (!(d.M > 0) || !std::isfinite(d.M)) return "M must be positive and finite";
    if (!(std::fabs(d.a) < d.M)) return "|a| must be below M";
    if (d.s < -2 || d.s > 2) return "s must be in [-2, 2]";
    if (d.n_r < 5 || d.n_theta < 5) return "n_r and n_theta must be >= 5";
    if (d.n_r > (1 << 22) || d.n_theta > (1 << 16) || (double)d.n_r * d.n_theta > 1.5e9)
        return "grid too large";
    if (!(d.rstar_max > d.rstar_min) || !std::isfinite(d.rstar_min) || !std::isfinite(d.rstar_max))
        return "need rstar_min < rstar_max, finite";
    if (!(d.dt > 0) || !std::isfinite(d.dt)) return "dt must be positive and finite";
    if (d.extract_every < 0 || d.wave_capacity < 0) return "extract_every and wave_capacity must be >= 0";
    if (!std::isfinite(d.rstar_obs)) return "rstar_obs must be finite";
    double h = (d.rstar_max - d.rstar_min) / (d.n_r - 1);
    long io = (long)std::floor((d.rstar_obs - d.rstar_min) / h + 0.5);
    if (io < 0 || io >= d.n_r) {
        std::snprintf(b, sizeof b, "rstar_obs %.17g outside the grid", d.rstar_obs);
        return b;
    }
    if (d.layer_start != 0.0) {
        const double R = d.layer_start;
        if (!std::isfinite(R) || !(R > 0.0) || !(R > d.rstar_min))
            return "layer_start must be finite, positive and above rstar_min";
        if (!(d.rstar_max - R >= 2.0 * h)) return "the layer needs at least two cells before rstar_max";
        if (d.s != -2) return "the hyperboloidal layer is for the s = -2 field";
    }
    return "";
}

// First output column whose stencil reaches into the layer (the half node
// i + 1/2 beyond rho = R); n_r for an instance without a layer.
int layer_first_column(const HostInst &h)
{
    const tk_instance_desc &d = h.desc;
    if (d.layer_start == 0.0) return d.n_r;
    int i = 0;
    while (i < d.n_r && !(d.rstar_min + (i + 0.5) * h.h > d.layer_start)) ++i;
    return i;
}

// Fused work list: strips of `cols` output columns (lanes i0 - halo ..
// i0 - halo + 63) x chunks of `rows` rows, longest first (waves are
// dispatched roughly in order).  rows == 0: whole strips, except that a
// strip whose lanes reach a hyperboloidal layer is cut into chunks of
// kLayerStripRows rows: the layer's waves take longer per row, and whole
// strips all run at once, so that they would set the pass's time.
void build_work(tk_ctx *c, int rows, int cols, int min_rows, int halo)
{
    c->work.clear();
    c->work_chunked = false;
    for (size_t k = 0; k < c->inst.size(); ++k) {
        const tk_instance_desc &d = c->inst[k].desc;
        const int iL = layer_first_column(c->inst[k]);
        for (int i0 = 0; i0 < d.n_r; i0 += cols) {
            // an instance ending in a hyperboloidal layer: its last strip
            // holds its last three columns, the null-infinity column and
            // the two it is extrapolated from (columns the strip shares
            // with the one before are written twice with equal values)
            const bool last = d.layer_start != 0.0 && i0 + cols >= d.n_r;
            const int s0 = last ? std::max(0, std::min(i0, d.n_r - 3)) : i0;
            const bool touch = d.layer_start != 0.0 && s0 - halo + 63 >= iL;
            const int rc = rows > 0 ? std::max(rows, min_rows) : touch ? kLayerStripRows : d.n_theta;
            for (int j0 = 0; j0 < d.n_theta; j0 += rc) {
                int j1 = std::min(d.n_theta, j0 + rc);
                // keep a pole chunk at least min_rows rows (the one-step pole
                // extrapolation needs rows 1, 2; a two-step chunk keeps four rows
                // from a pole it does not hold)
                if (d.n_theta - j1 > 0 && d.n_theta - j1 < min_rows) j1 = d.n_theta;
                c->work.push_back(WorkItem{(int)k, s0, j0, j1});
                c->work_chunked = c->work_chunked || j1 - j0 < d.n_theta;
                if (j1 == d.n_theta) break;
            }
        }
    }
    std::stable_sort(c->work.begin(), c->work.end(),
                     [](const WorkItem &x, const WorkItem &y) { return (x.j1 - x.j0) > (y.j1 - y.j0); });
    c->work_rows = rows;
    c->work_cols = cols;
}

// Strips of `cols` columns from column i0s to the end of instance k (or to
// i1), in chunks of `rows` rows (0 = whole columns); a chunk holding a pole
// row keeps at least three rows.
void push_strips(std::vector<WorkItem> &out, int k, const tk_instance_desc &d, int i0s, int i1, int cols, int rows)
{
    const int rc = rows > 0 ? rows : d.n_theta;
    for (int j0 = 0; j0 < d.n_theta; j0 += rc) {
        int j1 = std::min(d.n_theta, j0 + rc);
        if (d.n_theta - j1 > 0 && d.n_theta - j1 < 3) j1 = d.n_theta;
        for (int i0 = i0s; i0 < i1; i0 += cols) out.push_back(WorkItem{k, i0, j0, j1});
        if (j1 == d.n_theta) break;
    }
}

// Work list of the layer's two passes: strips of kLayerCols columns over
// whole instances in chunks of `rows` rows (0 = kLayerRows).
void build_layer_work(tk_ctx *c, int rows)
{
    c->lwork.clear();
    for (size_t k = 0; k < c->inst.size(); ++k)
        push_strips(c->lwork, (int)k, c->inst[k].desc, 0, c->inst[k].desc.n_r, kLayerCols, rows > 0 ? rows : kLayerRows);
    c->lwork_rows = rows;
}

size_t layer_work_capacity(const tk_ctx *c)
{
    size_t n = 0;  // chunks of at least 3 rows
    for (const HostInst &h : c->inst)
        n += (size_t)((h.desc.n_r + kLayerCols - 1) / kLayerCols) * (h.desc.n_theta / 3 + 1);
    return n;
}

size_t work_capacity(const tk_ctx *c)
{
    // upper bound over the shapes: chunks of 3 rows of kFusedCols-wide
    // strips, or chunks of 4 rows of kFused2Cols-wide strips
    size_t n = 0;
    for (const HostInst &h : c->inst) {
        size_t strips = (h.desc.n_r + kFusedCols - 1) / kFusedCols;
        size_t strips2 = (h.desc.n_r + kFused2Cols - 1) / kFused2Cols;
        n += std::max(strips * ((h.desc.n_theta + 2) / 3 + 1), strips2 * ((h.desc.n_theta + 3) / 4 + 1));
    }
    return n;
}

void layout(tk_ctx *c)
{
    size_t off = 0;
    const size_t A = 4096;
    c->off_ctl = off;
    off = align_up(off + sizeof(DevCtl), A);
    c->off_inst = off;
    off = align_up(off + c->inst.size() * sizeof(DevInst), A);
    c->off_blocks = off;
    off = align_up(off + c->blocks.size() * sizeof(int2), A);
    c->off_work = off;
    c->work_cap = work_capacity(c);
    off = align_up(off + c->work_cap * sizeof(WorkItem), A);
    c->off_linst = off;
    off = align_up(off + c->inst.size() * sizeof(LayerInst), A);
    c->off_lwork = off;
    c->lwork_cap = c->layered ? layer_work_capacity(c) : 0;
    off = align_up(off + c->lwork_cap * sizeof(WorkItem), A);
    c->off_lay.assign(c->inst.size(), 0);
    for (size_t k = 0; k < c->inst.size(); ++k) {
        if (c->inst[k].desc.layer_start == 0.0) continue;
        c->off_lay[k] = off;
        off = align_up(off + (size_t)(2 * c->inst[k].desc.n_r - 1) * sizeof(LayerTab), A);
    }
    for (HostInst &h : c->inst) {
        const tk_instance_desc &d = h.desc;
        size_t pts = (size_t)d.n_theta * h.pitch;
        h.off_rad = off;
        off = align_up(off + (size_t)(2 * d.n_r - 1) * sizeof(Radial), A);
        h.off_ang = off;
        off = align_up(off + (size_t)d.n_theta * sizeof(Angular), A);
        h.off_angf = off;
        off = align_up(off + (size_t)d.n_theta * sizeof(AngularF), A);
        size_t ubytes = c->prec == TK_FP64 ? pts * 32 : pts * 16;
        size_t cbytes = c->prec == TK_FP64 ? 0 : pts * 8;
        for (int b = 0; b < 2; ++b) {
            h.off_u[b] = off;
            off = align_up(off + ubytes, A);
            h.off_c[b] = off;
            off = align_up(off + cbytes, A);
        }
        h.off_half = off;
        off = align_up(off + (c->prec == TK_FP64 ? pts * 32 : 0), A);
        h.off_wave = off;
        off = align_up(off + (size_t)h.wave_cap * d.n_theta * 16, A);
    }
    c->need = off;
}

DevInst make_dev(const tk_ctx *c, size_t k)
{
    const HostInst &h = c->inst[k];
    DevInst D;
    std::memset(&D, 0, sizeof D);
    const tk_instance_desc &d = h.desc;
    D.n_r = d.n_r;
    D.n_theta = d.n_theta;
    D.pitch = h.pitch;
    D.m_even = (std::abs(d.m + d.s) % 2) == 0;  // pole rule: parity of m + s
    D.m = d.m;
    D.i_obs = h.i_obs;
    D.extract_every = d.extract_every;
    D.wave_cap = h.wave_cap;
    D.h = h.h;
    D.dth = h.dth;
    D.dt = d.dt;
    D.inv_h = 1.0 / h.h;
    D.inv_dth2 = 1.0 / (h.dth * h.dth);
    D.inv_2dth = 1.0 / (2.0 * h.dth);
    D.rstar_min = d.rstar_min;
    char *ws = c->ws;
    for (int b = 0; b < 2; ++b) {
        D.u[b] = ws + h.off_u[b];
        D.c[b] = ws + h.off_c[b];
    }
    D.half = ws + h.off_half;
    D.rad = (const Radial *)(ws + h.off_rad);
    D.ang = (const Angular *)(ws + h.off_ang);
    D.angf = (const AngularF *)(ws + h.off_angf);
    D.wave = (double *)(ws + h.off_wave);
    D.src_kind = h.src.kind;
    D.src_amp = h.src.amplitude;
    D.src_phase0 = h.src.phase0;
    D.src_Omega = h.src_Omega;
    D.src_rstar_p = h.src_rstar_p;
    D.src_sig_r = h.src.sigma_r_cells * h.h;
    D.src_sig_th = h.src.sigma_th_cells * h.dth;
    D.src_win = h.src.window_sigmas;
    D.src_t0 = h.src.t0;
    D.src_ramp_inv = h.src.ramp > 0.0 ? 1.0 / h.src.ramp : 0.0;
    D.a2 = d.a * d.a;
    D.kct = -2.0 * d.s * d.a;
    const bool lay = d.layer_start != 0.0 && k < c->off_lay.size();
    D.lay = lay ? ws + c->off_lay[k] : nullptr;
    D.lay_on = lay ? 1 : 0;
    D.lay_c0 = layer_first_column(h);
    return D;
}

// Whether a layered context steps with the layer kernels (the two-pass
// layer step, FP64) rather than with the marching kernels' layered form over
// whole instances (one and two steps a pass, both precisions).
bool layer_kernels(const tk_ctx *c, int kernel)
{
    return c->layered && kernel == TK_KERNEL_TWO_PASS;
}

int resolve_kernel(const tk_ctx *c)
{
    int k = c->tuning.kernel;
    if (k == TK_KERNEL_AUTO) k = c->tuning.rows_per_tile == 0 ? TK_KERNEL_FUSED2 : TK_KERNEL_FUSED;
    if (c->prec != TK_FP64 && k == TK_KERNEL_TWO_PASS) k = TK_KERNEL_FUSED;
    return k;
}

tk_status ensure_work(tk_ctx *c, int kernel)
{
    if (layer_kernels(c, kernel)) {
        const int rows = c->tuning.rows_per_tile;
        if (!c->lwork.empty() && c->lwork_rows == rows) return TK_OK;
        build_layer_work(c, rows);
        if (c->lwork.size() > c->lwork_cap) return fail(c, TK_E_STATE, "layer work list exceeds its reserved area");
        TK_HIP(c, hipMemcpyAsync(c->ws + c->off_lwork, c->lwork.data(), c->lwork.size() * sizeof(WorkItem),
                                 hipMemcpyHostToDevice, c->stream));
        TK_HIP(c, hipStreamSynchronize(c->stream));
        return TK_OK;
    }
    const int rows = c->tuning.rows_per_tile;
    const int cols = kernel == TK_KERNEL_FUSED2 ? kFused2Cols : kFusedCols;
    if (!c->work.empty() && c->work_rows == rows && c->work_cols == cols) return TK_OK;
    build_work(c, rows, cols, kernel == TK_KERNEL_FUSED2 ? 4 : 3, kernel == TK_KERNEL_FUSED2 ? 2 : 1);
    if (c->work.size() > c->work_cap) return fail(c, TK_E_STATE, "work list exceeds its reserved area");
    TK_HIP(c, hipMemcpyAsync(c->ws + c->off_work, c->work.data(), c->work.size() * sizeof(WorkItem),
                             hipMemcpyHostToDevice, c->stream));
    TK_HIP(c, hipStreamSynchronize(c->stream));
    return TK_OK;
}

// One launch advancing `steps` (1, or 2 with the two-step kernel) from step
// offset kstep, reading buffer (cur + kflip) & 1.
hipError_t launch_one(tk_ctx *c, int kernel, int steps, int kstep, int kflip)
{
    const DevInst *di = (const DevInst *)(c->ws + c->off_inst);
    const DevCtl *ctl = (const DevCtl *)(c->ws + c->off_ctl);
    if (layer_kernels(c, kernel))  // the layer's two passes
        return launch_layer(di, (const LayerInst *)(c->ws + c->off_linst), (int)c->inst.size(),
                            (const WorkItem *)(c->ws + c->off_lwork), (int)c->lwork.size(), ctl, kstep, kflip, c->stream);
    if (kernel == TK_KERNEL_TWO_PASS)
        return launch_two_pass(di, (const int2 *)(c->ws + c->off_blocks), (int)c->blocks.size(), ctl, kstep, kflip,
                               c->stream);
    const WorkItem *wk = (const WorkItem *)(c->ws + c->off_work);
    if (kernel == TK_KERNEL_TILED)
        return launch_tiled(c->prec == TK_FP64, di, wk, (int)c->work.size(), c->tuning.rows_per_tile, ctl, kstep,
                            kflip, (c->tuning.flags & TK_TUNE_NT_STORES) != 0, c->stream);
    FusedShape f;
    f.prefetch = c->tuning.prefetch_rows == 1 ? 1 : 3;
    f.nt = (c->tuning.flags & TK_TUNE_NT_STORES) != 0;
    f.waves = c->tuning.waves_per_simd == 0 ? 1 : c->tuning.waves_per_simd;
    f.two_step = steps == 2;
    f.chunked = c->work_chunked;
    return launch_fused(c->prec == TK_FP64, di, wk, (int)c->work.size(), c->work_cols, ctl, kstep, kflip, f,
                        c->stream, c->layered);
}

// The launches of n steps: pairs of steps with the two-step kernel, the
// rest one step at a time; then the control-block bump.  Returns the number
// of launches (buffer flips) in *flips.
tk_status enqueue_steps(tk_ctx *c, int kernel, long n, int *flips)
{
    long k = 0;
    int f = 0;
    if (kernel == TK_KERNEL_FUSED2) {
        for (; n - k >= 2; k += 2, ++f) {
            hipError_t e = launch_one(c, kernel, 2, (int)k, f & 1);
            if (e != hipSuccess) return fail(c, TK_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
        }
    }
    for (; k < n; ++k, ++f) {
        hipError_t e = launch_one(c, kernel, 1, (int)k, f & 1);
        if (e != hipSuccess) return fail(c, TK_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    hipError_t e = launch_bump((DevCtl *)(c->ws + c->off_ctl), (int)n, f & 1, c->stream);
    if (e != hipSuccess) return fail(c, TK_E_DEVICE, std::string("bump launch: ") + hipGetErrorString(e));
    *flips = f;
    return TK_OK;
}

void drop_graph(tk_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->g_steps = 0;
    c->g_kernel = -1;
    c->g_rows = -1;
    c->g_pf = -1;
    c->g_flags = -1;
    c->g_waves = -1;
}

tk_status ensure_graph(tk_ctx *c, int kernel, int G)
{
    if (c->gexec && c->g_steps == G && c->g_kernel == kernel && c->g_rows == c->tuning.rows_per_tile &&
        c->g_pf == c->tuning.prefetch_rows && c->g_flags == c->tuning.flags &&
        c->g_waves == c->tuning.waves_per_simd)
        return TK_OK;
    drop_graph(c);
    hipGraph_t g = nullptr;
    TK_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int flips = 0;
    tk_status st = enqueue_steps(c, kernel, G, &flips);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (st != TK_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(c, TK_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->gexec = nullptr;
        return fail(c, TK_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    c->g_steps = G;
    c->g_flips = flips;
    c->g_kernel = kernel;
    c->g_rows = c->tuning.rows_per_tile;
    c->g_pf = c->tuning.prefetch_rows;
    c->g_flags = c->tuning.flags;
    c->g_waves = c->tuning.waves_per_simd;
    c->counters.graphs_instantiated += 1;
    return TK_OK;
}

}  // namespace

extern "C" {

int tk_abi_version(void) { return TK_ABI_VERSION; }

const char *tk_last_error(const tk_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

tk_status tk_stable_dt(const tk_instance_desc *inst, double *dt_max)
{
    if (!inst || !dt_max) return fail(nullptr, TK_E_INVALID, "null argument");
    tk_instance_desc d = *inst;
    if (!(d.dt > 0) || !std::isfinite(d.dt)) d.dt = 1.0;  // the step itself is what is asked for
    std::string v = validate(d);
    if (!v.empty()) return fail(nullptr, TK_E_INVALID, v);
    *dt_max = stable_dt_bound(d);
    return TK_OK;
}

tk_status tk_init_grid(const tk_instance_desc *inst, int n_inst, tk_precision prec, void *hip_stream, tk_ctx **out)
{
    if (!inst || !out || n_inst <= 0) return fail(nullptr, TK_E_INVALID, "need instances and an output pointer");
    if (prec != TK_FP64 && prec != TK_FP32_COMP) return fail(nullptr, TK_E_INVALID, "unknown precision");
    tk_ctx *c = new (std::nothrow) tk_ctx();
    if (!c) return fail(nullptr, TK_E_NOMEM, "host allocation failed");
    c->prec = prec;
    c->stream = (hipStream_t)hip_stream;
    c->inst.resize(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        const tk_instance_desc &d = inst[k];
        std::string v = validate(d);
        if (!v.empty()) {
            delete c;
            return fail(nullptr, TK_E_INVALID, "instance " + std::to_string(k) + ": " + v);
        }
        double bound = stable_dt_bound(d);
        if (d.dt > bound * (1.0 + 1e-12) && !(d.flags & TK_FLAG_FORCE_DT)) {
            char b[256];
            std::snprintf(b, sizeof b, "instance %d: dt %.6g exceeds the stability bound %.6g", k, d.dt, bound);
            delete c;
            return fail(nullptr, TK_E_UNSTABLE, b);
        }
        HostInst &h = c->inst[k];
        std::memset(&h, 0, sizeof h);
        h.desc = d;
        h.src.kind = TK_SRC_NONE;
        h.h = (d.rstar_max - d.rstar_min) / (d.n_r - 1);
        h.dth = M_PI / (d.n_theta - 1);
        double q = std::sqrt((d.M - d.a) * (d.M + d.a));
        h.rp = d.M + q;
        h.rm = d.M - q;
        h.i_obs = (int)std::floor((d.rstar_obs - d.rstar_min) / h.h + 0.5);  // nearest node, ties up
        h.pitch = (d.n_r + 63) / 64 * 64;
        h.wave_cap = d.wave_capacity > 0 ? d.wave_capacity : 4096;
        h.wave_drained = 0;
        long long nb = ((long long)d.n_theta * d.n_r + 255) / 256;
        for (long long b = 0; b < nb; ++b) c->blocks.push_back(int2{k, (int)b});
    }
    if (c->blocks.size() > 0x7fffffff) {
        delete c;
        return fail(nullptr, TK_E_INVALID, "too many points");
    }
    for (int k = 0; k < n_inst; ++k) c->layered = c->layered || inst[k].layer_start != 0.0;
    layout(c);
    *out = c;
    return TK_OK;
}

tk_status tk_workspace_bytes(const tk_ctx *ctx, size_t *bytes)
{
    if (!ctx || !bytes) return fail(const_cast<tk_ctx *>(ctx), TK_E_INVALID, "null argument");
    *bytes = ctx->need;
    return TK_OK;
}

tk_status tk_bind_workspace(tk_ctx *c, void *dev_ptr, size_t bytes)
{
    if (!c || !dev_ptr) return fail(c, TK_E_INVALID, "null argument");
    if (c->ws) return fail(c, TK_E_STATE, "workspace already bound");
    if (bytes < c->need) return fail(c, TK_E_NOMEM, "workspace smaller than tk_workspace_bytes");
    if ((uintptr_t)dev_ptr % 256 != 0) return fail(c, TK_E_INVALID, "workspace must be 256-byte aligned");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, dev_ptr) != hipSuccess || attr.type != hipMemoryTypeDevice)
        return fail(c, TK_E_INVALID, "workspace is not device memory");
    if (!c->ev0) TK_HIP(c, hipEventCreate(&c->ev0));
    if (!c->ev1) TK_HIP(c, hipEventCreate(&c->ev1));
    c->device = attr.device;
    c->ws = (char *)dev_ptr;
    c->ws_bytes = bytes;
    tk_status st = TK_OK;
    // tables
    c->hdev.resize(c->inst.size());
    c->hrad.resize(c->inst.size());
    c->hang.resize(c->inst.size());
    c->hangf.resize(c->inst.size());
    for (size_t k = 0; k < c->inst.size() && st == TK_OK; ++k) {
        HostInst &h = c->inst[k];
        std::vector<Radial> &rad = c->hrad[k];
        std::vector<Angular> &ang = c->hang[k];
        std::vector<AngularF> &angf = c->hangf[k];
        rad.resize(2 * h.desc.n_r - 1);
        ang.resize(h.desc.n_theta);
        angf.resize(h.desc.n_theta);
        fill_radial(h, rad.data());
        fill_angular(h, ang.data());
        fill_source(h, rad.data(), ang.data());
        for (int j = 0; j < h.desc.n_theta; ++j)
            angf[j] = AngularF{(float)ang[j].sa, (float)ang[j].sn2, (float)ang[j].kcs, (float)ang[j].V2,
                               (float)ang[j].cot_h, 0.0f, 0.0f, 0.0f};
        c->hdev[k] = make_dev(c, k);
        hipError_t e = hipMemcpyAsync(c->ws + h.off_rad, rad.data(), rad.size() * sizeof(Radial),
                                      hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->ws + h.off_ang, ang.data(), ang.size() * sizeof(Angular), hipMemcpyHostToDevice,
                               c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->ws + h.off_angf, angf.data(), angf.size() * sizeof(AngularF),
                               hipMemcpyHostToDevice, c->stream);
        std::vector<LayerTab> lay;
        if (e == hipSuccess && h.desc.layer_start != 0.0) {
            lay.resize(2 * h.desc.n_r - 1);
            fill_layer(h, lay.data());
            e = hipMemcpyAsync(c->ws + c->off_lay[k], lay.data(), lay.size() * sizeof(LayerTab),
                               hipMemcpyHostToDevice, c->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) st = fail(c, TK_E_DEVICE, std::string("table upload: ") + hipGetErrorString(e));
    }
    if (st == TK_OK) {
        std::vector<LayerInst> li(c->inst.size());
        for (size_t k = 0; k < c->inst.size(); ++k) {
            const bool on = c->inst[k].desc.layer_start != 0.0;
            li[k] = LayerInst{on ? (const LayerTab *)(c->ws + c->off_lay[k]) : nullptr, on ? 1 : 0};
        }
        hipError_t e = hipMemcpyAsync(c->ws + c->off_linst, li.data(), li.size() * sizeof(LayerInst),
                                      hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) st = fail(c, TK_E_DEVICE, std::string("layer upload: ") + hipGetErrorString(e));
    }
    if (st == TK_OK) {
        // zero everything after the tables: fields, compensation, half array, rings, control
        hipError_t e = hipMemsetAsync(c->ws + c->off_ctl, 0, sizeof(DevCtl), c->stream);
        for (size_t k = 0; k < c->inst.size() && e == hipSuccess; ++k) {
            const HostInst &h = c->inst[k];
            e = hipMemsetAsync(c->ws + h.off_u[0], 0, h.off_wave - h.off_u[0], c->stream);
            if (e == hipSuccess)
                e = hipMemsetAsync(c->ws + h.off_wave, 0, (size_t)h.wave_cap * h.desc.n_theta * 16, c->stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->ws + c->off_inst, c->hdev.data(), c->hdev.size() * sizeof(DevInst),
                               hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(c->ws + c->off_blocks, c->blocks.data(), c->blocks.size() * sizeof(int2),
                               hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) st = fail(c, TK_E_DEVICE, std::string("workspace init: ") + hipGetErrorString(e));
    }
    if (st == TK_OK) st = ensure_work(c, TK_KERNEL_FUSED);
    if (st != TK_OK) {
        c->ws = nullptr;
        c->ws_bytes = 0;
        return st;
    }
    c->step = 0;
    c->cur = 0;
    return TK_OK;
}

static tk_status check_inst(tk_ctx *c, int inst)
{
    if (!c) return TK_E_INVALID;
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, TK_E_INVALID, "instance index out of range");
    if (!c->ws) return fail(c, TK_E_STATE, "no workspace bound");
    return TK_OK;
}

// FP32-compensated storage: value = f + c with f = fp32(x), c = bf16(x - f).
static inline uint16_t bf16_rne(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
static inline float bf16_to_f(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

tk_status tk_set_fields(tk_ctx *c, int inst, const double *phi, const double *pi)
{
    tk_status st = check_inst(c, inst);
    if (st != TK_OK) return st;
    if (!phi || !pi) return fail(c, TK_E_INVALID, "null field pointer");
    const HostInst &h = c->inst[inst];
    const int nr = h.desc.n_r, nt = h.desc.n_theta, p = h.pitch;
    const int cur = c->cur;
    if (c->prec == TK_FP64) {
        std::vector<double> buf((size_t)nt * p * 4, 0.0);
        for (int j = 0; j < nt; ++j)
            for (int i = 0; i < nr; ++i) {
                size_t s = ((size_t)j * nr + i) * 2, d = ((size_t)j * p + i) * 4;
                buf[d + 0] = phi[s];
                buf[d + 1] = phi[s + 1];
                buf[d + 2] = pi[s];
                buf[d + 3] = pi[s + 1];
            }
        TK_HIP(c, hipMemcpyAsync(c->ws + h.off_u[cur], buf.data(), buf.size() * sizeof(double),
                                 hipMemcpyHostToDevice, c->stream));
        TK_HIP(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> fb((size_t)nt * p * 4, 0.0f);
        std::vector<uint16_t> cb((size_t)nt * p * 4, 0);
        for (int j = 0; j < nt; ++j)
            for (int i = 0; i < nr; ++i) {
                size_t s = ((size_t)j * nr + i) * 2, d = ((size_t)j * p + i) * 4;
                const double v[4] = {phi[s], phi[s + 1], pi[s], pi[s + 1]};
                for (int q = 0; q < 4; ++q) {
                    float f = (float)v[q];
                    fb[d + q] = f;
                    cb[d + q] = bf16_rne((float)(v[q] - (double)f));
                }
            }
        TK_HIP(c, hipMemcpyAsync(c->ws + h.off_u[cur], fb.data(), fb.size() * sizeof(float), hipMemcpyHostToDevice,
                                 c->stream));
        TK_HIP(c, hipMemcpyAsync(c->ws + h.off_c[cur], cb.data(), cb.size() * sizeof(uint16_t),
                                 hipMemcpyHostToDevice, c->stream));
        TK_HIP(c, hipStreamSynchronize(c->stream));
    }
    return TK_OK;
}

tk_status tk_get_fields(tk_ctx *c, int inst, double *phi, double *pi)
{
    tk_status st = check_inst(c, inst);
    if (st != TK_OK) return st;
    if (!phi || !pi) return fail(c, TK_E_INVALID, "null field pointer");
    const HostInst &h = c->inst[inst];
    const int nr = h.desc.n_r, nt = h.desc.n_theta, p = h.pitch;
    const int cur = c->cur;
    if (c->prec == TK_FP64) {
        std::vector<double> buf((size_t)nt * p * 4);
        TK_HIP(c, hipMemcpyAsync(buf.data(), c->ws + h.off_u[cur], buf.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream));
        TK_HIP(c, hipStreamSynchronize(c->stream));
        for (int j = 0; j < nt; ++j)
            for (int i = 0; i < nr; ++i) {
                size_t d = ((size_t)j * nr + i) * 2, s = ((size_t)j * p + i) * 4;
                phi[d] = buf[s];
                phi[d + 1] = buf[s + 1];
                pi[d] = buf[s + 2];
                pi[d + 1] = buf[s + 3];
            }
    } else {
        std::vector<float> fb((size_t)nt * p * 4);
        std::vector<uint16_t> cb((size_t)nt * p * 4);
        TK_HIP(c, hipMemcpyAsync(fb.data(), c->ws + h.off_u[cur], fb.size() * sizeof(float), hipMemcpyDeviceToHost,
                                 c->stream));
        TK_HIP(c, hipMemcpyAsync(cb.data(), c->ws + h.off_c[cur], cb.size() * sizeof(uint16_t),
                                 hipMemcpyDeviceToHost, c->stream));
        TK_HIP(c, hipStreamSynchronize(c->stream));
        for (int j = 0; j < nt; ++j)
            for (int i = 0; i < nr; ++i) {
                size_t d = ((size_t)j * nr + i) * 2, s = ((size_t)j * p + i) * 4;
                double v[4];
                for (int q = 0; q < 4; ++q) v[q] = (double)fb[s + q] + (double)bf16_to_f(cb[s + q]);
                phi[d] = v[0];
                phi[d + 1] = v[1];
                pi[d] = v[2];
                pi[d + 1] = v[3];
            }
    }
    return TK_OK;
}

tk_status tk_set_source(tk_ctx *c, int inst, const tk_source_desc *src)
{
    tk_status st = check_inst(c, inst);
    if (st != TK_OK) return st;
    if (!src) return fail(c, TK_E_INVALID, "null source");
    HostInst &h = c->inst[inst];
    tk_source_desc s = *src;
    double Om = 0.0, rsp = 0.0;
    if (s.kind == TK_SRC_CIRCULAR_GAUSSIAN || s.kind == TK_SRC_CIRCULAR_STEP_DELTA ||
        s.kind == TK_SRC_CIRCULAR_LINEAR_DELTA) {
        if (!(s.r0 > h.rp) || !std::isfinite(s.r0)) return fail(c, TK_E_INVALID, "r0 must lie outside the horizon");
        if (!std::isfinite(s.amplitude) || !std::isfinite(s.phase0) || !std::isfinite(s.t0))
            return fail(c, TK_E_INVALID, "source amplitude, phase and t0 must be finite");
        if (!(s.ramp >= 0.0) || !std::isfinite(s.ramp))
            return fail(c, TK_E_INVALID, "source ramp must be finite and >= 0");
        if (s.kind == TK_SRC_CIRCULAR_GAUSSIAN &&
            (!(s.sigma_r_cells > 0) || !(s.sigma_th_cells > 0) || !(s.window_sigmas > 0) ||
             !std::isfinite(s.sigma_r_cells) || !std::isfinite(s.sigma_th_cells) || !std::isfinite(s.window_sigmas)))
            return fail(c, TK_E_INVALID, "source widths and window must be positive and finite");
        Om = orbit_frequency(h.desc.M, h.desc.a, s.r0);
        rsp = tortoise_of_x(h.desc.M, h.desc.a, s.r0 - h.rp);
        if (h.desc.layer_start != 0.0) {
            const double reach = s.kind == TK_SRC_CIRCULAR_GAUSSIAN ? s.window_sigmas * s.sigma_r_cells * h.h : 2.0 * h.h;
            if (!(rsp + reach < h.desc.layer_start))
                return fail(c, TK_E_INVALID, "the source must lie below the hyperboloidal layer");
        }
    } else if (s.kind != TK_SRC_NONE) {
        return fail(c, TK_E_INVALID, "unknown source kind");
    }
    h.src = s;
    h.src_Omega = Om;
    h.src_rstar_p = rsp;
    c->hdev[inst] = make_dev(c, (size_t)inst);
    fill_source(h, c->hrad[inst].data(), c->hang[inst].data());
    TK_HIP(c, hipMemcpyAsync(c->ws + h.off_rad, c->hrad[inst].data(), c->hrad[inst].size() * sizeof(Radial),
                             hipMemcpyHostToDevice, c->stream));
    TK_HIP(c, hipMemcpyAsync(c->ws + h.off_ang, c->hang[inst].data(), c->hang[inst].size() * sizeof(Angular),
                             hipMemcpyHostToDevice, c->stream));
    TK_HIP(c, hipMemcpyAsync(c->ws + c->off_inst + inst * sizeof(DevInst), &c->hdev[inst], sizeof(DevInst),
                             hipMemcpyHostToDevice, c->stream));
    TK_HIP(c, hipStreamSynchronize(c->stream));
    return TK_OK;
}

tk_status tk_step(tk_ctx *c, long n_steps)
{
    if (!c) return TK_E_INVALID;
    if (n_steps < 0 || n_steps > (1L << 40)) return fail(c, TK_E_INVALID, "n_steps out of range");
    if (!c->ws) return fail(c, TK_E_STATE, "no workspace bound");
    if (n_steps == 0) return TK_OK;
    const int G = c->tuning.graph_steps;
    if (G > 0 && c->stream == nullptr)
        return fail(c, TK_E_STATE, "graph_steps > 0 needs a stream other than the NULL stream (it cannot be captured)");
    const int kernel = resolve_kernel(c);
    if (kernel != TK_KERNEL_TWO_PASS || c->layered) {
        tk_status st = ensure_work(c, kernel);
        if (st != TK_OK) return st;
    }
    long left = n_steps;
    if (G > 0 && left >= G) {
        tk_status st = ensure_graph(c, kernel, G);
        if (st != TK_OK) return st;
        while (left >= G) {
            TK_HIP(c, hipGraphLaunch(c->gexec, c->stream));
            left -= G;
            c->step += G;
            c->cur = (c->cur + c->g_flips) & 1;
            c->counters.graph_launches += 1;
        }
    }
    while (left > 0) {
        long chunk = std::min(left, 1L << 20);
        int flips = 0;
        tk_status st = enqueue_steps(c, kernel, chunk, &flips);
        if (st != TK_OK) return st;
        left -= chunk;
        c->step += chunk;
        c->cur = (c->cur + flips) & 1;
        c->counters.eager_launches += flips + 1;  // the step launches and the control-block bump
    }
    return TK_OK;
}

tk_status tk_prepare(tk_ctx *c, long n_steps)
{
    if (!c) return TK_E_INVALID;
    if (n_steps < 0 || n_steps > (1L << 40)) return fail(c, TK_E_INVALID, "n_steps out of range");
    if (!c->ws) return fail(c, TK_E_STATE, "no workspace bound");
    const int kernel = resolve_kernel(c);
    if (kernel != TK_KERNEL_TWO_PASS || c->layered) {
        tk_status st = ensure_work(c, kernel);
        if (st != TK_OK) return st;
    }
    const int G = c->tuning.graph_steps;
    if (G > 0 && c->stream == nullptr)
        return fail(c, TK_E_STATE, "graph_steps > 0 needs a stream other than the NULL stream (it cannot be captured)");
    if (G > 0 && n_steps >= G) return ensure_graph(c, kernel, G);
    return TK_OK;
}

tk_status tk_get_counters(const tk_ctx *c, tk_counters *out)
{
    if (!c || !out) return TK_E_INVALID;
    *out = c->counters;
    return TK_OK;
}

tk_status tk_extract(tk_ctx *c, int inst, double *out, long max_samples, long *n_samples)
{
    tk_status st = check_inst(c, inst);
    if (st != TK_OK) return st;
    if (!n_samples || (max_samples > 0 && !out) || max_samples < 0) return fail(c, TK_E_INVALID, "bad output");
    HostInst &h = c->inst[inst];
    *n_samples = 0;
    const int K = h.desc.extract_every;
    if (K <= 0) return TK_OK;
    const long long produced = c->step / K;
    const long long pending = produced - h.wave_drained;
    if (pending > h.wave_cap) {
        char b[200];
        std::snprintf(b, sizeof b, "waveform ring overrun: %lld samples since the last extract, capacity %d",
                      pending, h.wave_cap);
        return fail(c, TK_E_STATE, b);
    }
    const long long cnt = std::min<long long>(pending, max_samples);
    const size_t row = (size_t)h.desc.n_theta * 2;
    long long done = 0;
    while (done < cnt) {
        long long k0 = h.wave_drained + done;
        long long slot = k0 % h.wave_cap;
        long long run = std::min<long long>(cnt - done, h.wave_cap - slot);
        TK_HIP(c, hipMemcpyAsync(out + (size_t)done * row, c->ws + h.off_wave + (size_t)slot * row * sizeof(double),
                                 (size_t)run * row * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        done += run;
    }
    TK_HIP(c, hipStreamSynchronize(c->stream));
    h.wave_drained += cnt;
    *n_samples = (long)cnt;
    if (!finite_all(out, (size_t)cnt * row)) return fail(c, TK_E_NONFINITE, "non-finite waveform sample");
    return TK_OK;
}

tk_status tk_get_step(const tk_ctx *c, long *step)
{
    if (!c || !step) return TK_E_INVALID;
    *step = (long)c->step;
    return TK_OK;
}

tk_status tk_set_step(tk_ctx *c, long step)
{
    if (!c) return TK_E_INVALID;
    if (step < 0) return fail(c, TK_E_INVALID, "step must be >= 0");
    if (!c->ws) return fail(c, TK_E_STATE, "no workspace bound");
    TK_HIP(c, hipStreamSynchronize(c->stream));
    // the state stays where it is; only the time index changes
    DevCtl ctl;
    std::memset(&ctl, 0, sizeof ctl);
    ctl.step = step;
    ctl.cur = c->cur;
    TK_HIP(c, hipMemcpyAsync(c->ws + c->off_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, c->stream));
    TK_HIP(c, hipStreamSynchronize(c->stream));
    c->step = step;
    for (HostInst &h : c->inst) h.wave_drained = h.desc.extract_every > 0 ? step / h.desc.extract_every : 0;
    return TK_OK;
}

tk_status tk_set_tuning(tk_ctx *c, const tk_tuning *t)
{
    if (!c || !t) return TK_E_INVALID;
    if (t->kernel < TK_KERNEL_AUTO || t->kernel > TK_KERNEL_TILED)
        return fail(c, TK_E_INVALID, "unknown kernel");
    if (t->kernel == TK_KERNEL_TILED && t->rows_per_tile != 4 && t->rows_per_tile != 8)
        return fail(c, TK_E_INVALID, "the tiled kernel takes rows_per_tile 4 or 8");
    if (t->kernel == TK_KERNEL_FUSED2 && t->rows_per_tile != 0 && t->rows_per_tile < 4)
        return fail(c, TK_E_INVALID, "the two-step kernel takes whole strips (rows_per_tile 0) or chunks of >= 4 rows");
    if (t->kernel == TK_KERNEL_TWO_PASS && c->prec != TK_FP64)
        return fail(c, TK_E_INVALID, "the two-pass kernel is FP64 only");
    if (c->layered && t->kernel == TK_KERNEL_TILED)
        return fail(c, TK_E_INVALID, "the tiled kernel has no hyperboloidal layer form");
    if (t->rows_per_tile < 0 || (t->rows_per_tile > 0 && t->rows_per_tile < 3))
        return fail(c, TK_E_INVALID, "rows_per_tile must be 0 or >= 3");
    if (t->graph_steps < 0 || t->graph_steps > 100000) return fail(c, TK_E_INVALID, "graph_steps out of range");
    if (t->graph_steps > 0 && c->stream == nullptr)
        return fail(c, TK_E_INVALID, "graph_steps > 0 needs a stream other than the NULL stream (it cannot be captured)");
    if (t->prefetch_rows != 0 && t->prefetch_rows != 1 && t->prefetch_rows != 3)
        return fail(c, TK_E_INVALID, "prefetch_rows must be 0, 1 or 3");
    if (t->flags & ~TK_TUNE_NT_STORES) return fail(c, TK_E_INVALID, "unknown tuning flags");
    {
        const int pf = t->prefetch_rows == 0 ? 3 : t->prefetch_rows;
        const bool nt = (t->flags & TK_TUNE_NT_STORES) != 0;
        (void)pf;
        (void)nt;
        if (t->waves_per_simd != 0)
            return fail(c, TK_E_INVALID, "waves_per_simd must be 0 (forced-occupancy shapes are not compiled)");
    }
    c->tuning = *t;
    if (c->tuning.prefetch_rows == 0) c->tuning.prefetch_rows = 3;
    if (c->ws && (resolve_kernel(c) != TK_KERNEL_TWO_PASS || c->layered)) {
        tk_status st = ensure_work(c, resolve_kernel(c));
        if (st != TK_OK) return st;
    }
    return TK_OK;
}

tk_status tk_get_tuning(const tk_ctx *c, tk_tuning *t)
{
    if (!c || !t) return TK_E_INVALID;
    *t = c->tuning;
    return TK_OK;
}

// What a run of steps changes, which the autotuner saves and restores: the
// current state (and its compensation terms), the waveform rings and the
// control block.  Each span is placed at a 256-byte aligned offset of the
// save area.
struct SaveSpan {
    size_t off, bytes, save;
};
static std::vector<SaveSpan> autotune_spans(const tk_ctx *c, size_t *total)
{
    std::vector<SaveSpan> spans;
    size_t t = 0;
    auto add = [&](size_t off, size_t bytes) {
        spans.push_back(SaveSpan{off, bytes, t});
        t += align_up(bytes, 256);
    };
    for (const HostInst &h : c->inst) {
        const size_t pts = (size_t)h.desc.n_theta * h.pitch;
        add(h.off_u[c->cur], c->prec == TK_FP64 ? pts * 32 : pts * 16);
        if (c->prec != TK_FP64) add(h.off_c[c->cur], pts * 8);
        add(h.off_wave, (size_t)h.wave_cap * h.desc.n_theta * 16);
    }
    add(c->off_ctl, sizeof(DevCtl));
    *total = t;
    return spans;
}

tk_status tk_autotune_bytes(const tk_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return TK_E_INVALID;
    (void)autotune_spans(c, bytes);
    return TK_OK;
}

// Rows per chunk that fill the device with two-step waves when whole strips
// do not: the smallest chunks (at least 4 rows) that keep the work list
// within one wave per slot at two waves per SIMD, so that all of it runs at
// once with the least halo recomputed; 0 when whole strips already give at
// least that many waves.
static int fill_rows(const tk_ctx *c)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus <= 0)
        return 0;
    const long slots = 2L * 4L * cus;
    long strips = 0;
    int nt_max = 0;
    for (const HostInst &h : c->inst) {
        strips += (h.desc.n_r + kFused2Cols - 1) / kFused2Cols;
        nt_max = std::max(nt_max, h.desc.n_theta);
    }
    if (strips <= 0 || strips >= slots) return 0;
    const long per = slots / strips;  // chunks per strip
    if (per < 2) return 0;
    const int rows = (int)((nt_max + per - 1) / per);
    return rows >= 4 && rows < nt_max ? rows : 0;
}

// Time every candidate launch shape on the context's own instances and keep
// the fastest; the state, step counter and waveform rings are saved to `save`
// (device memory of at least the spans' total) and restored afterwards.
static tk_status autotune_run(tk_ctx *c, int warmup, int steps, char *save, const std::vector<SaveSpan> &spans,
                              double *best_ms_per_step, int *n_tried)
{
    warmup += warmup & 1;
    steps += steps & 1;
    TK_HIP(c, hipStreamSynchronize(c->stream));
    hipError_t e = hipSuccess;
    for (const SaveSpan &sp : spans)
        if (e == hipSuccess)
            e = hipMemcpyAsync(save + sp.save, c->ws + sp.off, sp.bytes, hipMemcpyDeviceToDevice, c->stream);
    hipEvent_t e0 = c->ev0, e1 = c->ev1;

    const tk_tuning keep = c->tuning;
    const long long step0 = c->step;
    const int cur0 = c->cur;
    drop_graph(c);
    // candidates: every compiled fused shape with the two-step and the
    // one-step kernels (whole strips, or chunks of rows, which give a small
    // workload more waves), the tiled kernel (short tiles for small grids),
    // and the two-pass kernel (FP64)
    const int shapes[][3] = {{3, 1, 0}, {3, 0, 0}, {1, 1, 0}, {1, 0, 0}};
    std::vector<tk_tuning> cand;
    std::vector<int> rows2 = {0, 32, 16};
    const int fill = fill_rows(c);
    if (fill > 0 && fill != 16 && fill != 32) rows2.push_back(fill);
    for (int rows : rows2)
        for (const auto &sh : shapes)
            cand.push_back(tk_tuning{TK_KERNEL_FUSED2, rows, 0, sh[0], sh[1] ? TK_TUNE_NT_STORES : 0, sh[2]});
    for (int rows : {0, 64, 16})
        for (const auto &sh : shapes)
            cand.push_back(tk_tuning{TK_KERNEL_FUSED, rows, 0, sh[0], sh[1] ? TK_TUNE_NT_STORES : 0, sh[2]});
    for (int rows : {8, 4})
        for (int ntf : {(int)TK_TUNE_NT_STORES, 0}) cand.push_back(tk_tuning{TK_KERNEL_TILED, rows, 0, 3, ntf, 0});
    if (c->prec == TK_FP64) cand.push_back(tk_tuning{TK_KERNEL_TWO_PASS, 0, 0, 3, TK_TUNE_NT_STORES, 0});
    if (c->layered) {
        cand.clear();
        // the layered marching kernels (one u^n row in flight), and the
        // layer's two-pass step (FP64)
        for (int rows : {0, 32, 16})
            for (int ntf : {(int)TK_TUNE_NT_STORES, 0}) cand.push_back(tk_tuning{TK_KERNEL_FUSED2, rows, 0, 1, ntf, 0});
        for (int rows : {0, 64, 16}) cand.push_back(tk_tuning{TK_KERNEL_FUSED, rows, 0, 1, TK_TUNE_NT_STORES, 0});
        if (c->prec == TK_FP64)
            for (int rows : {0, 32}) cand.push_back(tk_tuning{TK_KERNEL_TWO_PASS, rows, 0, 3, TK_TUNE_NT_STORES, 0});
    }

    tk_status st = e == hipSuccess ? TK_OK : fail(c, TK_E_DEVICE, std::string("autotune setup: ") + hipGetErrorString(e));
    // two passes over the candidates in opposite orders, each candidate's
    // faster time counting: one pass was biased by the order of timing (the
    // shapes timed late came out ahead of faster ones timed early)
    std::vector<double> t_best(cand.size(), 1e300);
    for (int pass = 0; pass < 2 && st == TK_OK; ++pass) {
        for (size_t q = 0; q < cand.size(); ++q) {
            const size_t i = pass == 0 ? q : cand.size() - 1 - q;
            c->tuning = cand[i];
            const int kernel = resolve_kernel(c);
            if (kernel != TK_KERNEL_TWO_PASS || c->layered) st = ensure_work(c, kernel);
            int flips = 0;
            if (st == TK_OK && warmup > 0) st = enqueue_steps(c, kernel, warmup, &flips);
            if (st == TK_OK && (e = hipEventRecord(e0, c->stream)) != hipSuccess)
                st = fail(c, TK_E_DEVICE, std::string("autotune event: ") + hipGetErrorString(e));
            if (st == TK_OK) st = enqueue_steps(c, kernel, steps, &flips);
            if (st == TK_OK && (e = hipEventRecord(e1, c->stream)) != hipSuccess)
                st = fail(c, TK_E_DEVICE, std::string("autotune event: ") + hipGetErrorString(e));
            float ms = 0.0f;
            if (st == TK_OK &&
                ((e = hipEventSynchronize(e1)) != hipSuccess || (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess))
                st = fail(c, TK_E_DEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
            if (st != TK_OK) break;
            t_best[i] = std::min(t_best[i], (double)ms / steps);
        }
    }
    double best = 1e300;
    tk_tuning best_t = keep;
    const int tried = (int)cand.size();
    for (size_t i = 0; i < cand.size(); ++i)
        if (t_best[i] < best) {
            best = t_best[i];
            best_t = cand[i];
        }
    // restore the simulation as it was
    hipError_t er = hipStreamSynchronize(c->stream);
    for (const SaveSpan &sp : spans)
        if (er == hipSuccess)
            er = hipMemcpyAsync(c->ws + sp.off, save + sp.save, sp.bytes, hipMemcpyDeviceToDevice, c->stream);
    if (er == hipSuccess) er = hipStreamSynchronize(c->stream);
    c->step = step0;
    c->cur = cur0;
    if (er != hipSuccess && st == TK_OK) st = fail(c, TK_E_DEVICE, std::string("autotune restore: ") + hipGetErrorString(er));
    if (st != TK_OK) {
        c->tuning = keep;
        return st;
    }
    best_t.graph_steps = keep.graph_steps;
    c->tuning = best_t;
    if (resolve_kernel(c) != TK_KERNEL_TWO_PASS || c->layered) {
        st = ensure_work(c, resolve_kernel(c));
        if (st != TK_OK) return st;
    }
    if (best_ms_per_step) *best_ms_per_step = best;
    if (n_tried) *n_tried = tried;
    return TK_OK;
}

static tk_status autotune_args(tk_ctx *c, int warmup, int steps)
{
    if (!c) return TK_E_INVALID;
    if (!c->ws) return fail(c, TK_E_STATE, "no workspace bound");
    if (warmup < 0 || warmup > 100000 || steps < 1 || steps > 100000)
        return fail(c, TK_E_INVALID, "warmup must be in [0, 1e5] and steps in [1, 1e5]");
    return TK_OK;
}

tk_status tk_autotune(tk_ctx *c, int warmup, int steps, void *save_area, size_t save_bytes,
                      double *best_ms_per_step, int *n_tried)
{
    tk_status st = autotune_args(c, warmup, steps);
    if (st != TK_OK) return st;
    size_t total = 0;
    const std::vector<SaveSpan> spans = autotune_spans(c, &total);
    if (!save_area) return fail(c, TK_E_INVALID, "autotune: null save area");
    if ((uintptr_t)save_area % 256 != 0) return fail(c, TK_E_INVALID, "autotune: save area must be 256-byte aligned");
    if (save_bytes < total) return fail(c, TK_E_NOMEM, "autotune: save area smaller than tk_autotune_bytes");
    {
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, save_area) != hipSuccess || attr.type != hipMemoryTypeDevice) {
            (void)hipGetLastError();
            return fail(c, TK_E_INVALID, "autotune: save area is not device memory");
        }
    }
    return autotune_run(c, warmup, steps, (char *)save_area, spans, best_ms_per_step, n_tried);
}

tk_status tk_autotune_static(tk_ctx *c, int warmup, int steps, double *best_ms_per_step, int *n_tried)
{
    tk_status st = autotune_args(c, warmup, steps);
    if (st != TK_OK) return st;
    size_t total = 0;
    const std::vector<SaveSpan> spans = autotune_spans(c, &total);
    if (total > kScratchBytes) {
        char b[256];
        std::snprintf(b, sizeof b,
                      "autotune_static: the context's save area needs %zu bytes, more than the %zu bytes of the "
                      "static scratch area (use tk_autotune with a caller save area)",
                      total, kScratchBytes);
        return fail(c, TK_E_NOMEM, b);
    }
    static_assert(kScratchBytes == (size_t)TK_AUTOTUNE_STATIC_MAX_BYTES, "the header states the scratch size");
    std::lock_guard<std::mutex> g(scratch_user_lock());
    void *area = nullptr;
    const hipError_t e = scratch_area(c->device, &area);
    if (e != hipSuccess) return fail(c, TK_E_DEVICE, std::string("autotune_static: scratch area: ") + hipGetErrorString(e));
    return autotune_run(c, warmup, steps, (char *)area, spans, best_ms_per_step, n_tried);
}

tk_status tk_synchronize(tk_ctx *c)
{
    if (!c) return TK_E_INVALID;
    TK_HIP(c, hipStreamSynchronize(c->stream));
    return TK_OK;
}

tk_status tk_destroy(tk_ctx *c)
{
    if (!c) return TK_E_INVALID;
    if (c->ws) (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
    return TK_OK;
}

}  // extern "C"
