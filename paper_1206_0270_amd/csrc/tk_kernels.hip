// HIP kernels of the Teukolsky m-mode stepper (gfx950).
//
// A step is the two-step Lax-Wendroff scheme of Eqs. (3)-(4) with the pole
// and radial conditions of Section 2.2 applied after each step.  Fields are
// stored per point as (Phi.re, Phi.im, Pi.re, Pi.im) on rows of constant
// theta (r* contiguous), so a wavefront's 64 lanes read 64 consecutive r*
// points: 2 KB per row per access in FP64.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "tk_device.h"
#include "tk_kernels.h"
#include "tk_layer.h"

namespace tk {

// ---------------------------------------------------------------------------
// Two-pass form: Eq. (3) into a half-step array in HBM, then Eq. (4).
// One thread per point; kept as a simple, independent check of the fused
// kernel and as a fallback launch shape.
// ---------------------------------------------------------------------------

__device__ __forceinline__ P4 stage1_at(const DevInst &I, const double4 *u, int i, int j, double t)
{
    // half node i+1/2, row j (1 <= j <= n_theta - 2)
    const int p = I.pitch;
    const P4 a0 = ld_p4(u + (size_t)j * p + i), a1 = ld_p4(u + (size_t)j * p + i + 1);
    const P4 am0 = ld_p4(u + (size_t)(j - 1) * p + i), am1 = ld_p4(u + (size_t)(j - 1) * p + i + 1);
    const P4 ap0 = ld_p4(u + (size_t)(j + 1) * p + i), ap1 = ld_p4(u + (size_t)(j + 1) * p + i + 1);
    const P4 bar = half_sum(a1, a0);
    const cd phm = half_sum(am1, am0).phi, php = half_sum(ap1, ap0).phi;
    const Radial R = load_entry(gload_ptr(I.rad) + (2 * i + 1));
    const Angular A = load_entry(gload_ptr(I.ang) + (j));
    const Coef c = coef_at(R, A);
    const cd F = R.srcg * A.srcg != 0.0 ? source_value(R.srcg, A.srcg, source_phase(I, t)) : mk(0, 0);
    return lw_point(c, bar, phm, bar.phi, php, bar.pi, a1 - a0, 0.5 * I.dt, I.inv_h, I.inv_dth2, I.inv_2dth, F);
}

__device__ __forceinline__ P4 stage2_at(const DevInst &I, const double4 *u, const double4 *hf, int i, int j, double t)
{
    // node i, row j (1 <= i <= n_r - 2, 1 <= j <= n_theta - 2); hf[.][i] is i+1/2
    const int p = I.pitch;
    const P4 h0 = ld_p4(hf + (size_t)j * p + i - 1), h1 = ld_p4(hf + (size_t)j * p + i);
    const P4 hm0 = ld_p4(hf + (size_t)(j - 1) * p + i - 1), hm1 = ld_p4(hf + (size_t)(j - 1) * p + i);
    const P4 hp0 = ld_p4(hf + (size_t)(j + 1) * p + i - 1), hp1 = ld_p4(hf + (size_t)(j + 1) * p + i);
    const P4 til = half_sum(h1, h0);
    const cd phm = half_sum(hm1, hm0).phi, php = half_sum(hp1, hp0).phi;
    const Radial R = load_entry(gload_ptr(I.rad) + (2 * i));
    const Angular A = load_entry(gload_ptr(I.ang) + (j));
    const Coef c = coef_at(R, A);
    const cd F = R.srcg * A.srcg != 0.0 ? source_value(R.srcg, A.srcg, source_phase(I, t)) : mk(0, 0);
    const P4 un = ld_p4(u + (size_t)j * p + i);
    return lw_point(c, un, phm, til.phi, php, til.pi, h1 - h0, I.dt, I.inv_h, I.inv_dth2, I.inv_2dth, F);
}

__global__ void __launch_bounds__(256) k_two_pass_half(const DevInst *__restrict__ insts, const int2 *__restrict__ blocks,
                                                       const DevCtl *__restrict__ ctl, int kstep, int kflip)
{
    const int2 bl = blocks[blockIdx.x];
    const DevInst &I = insts[bl.x];
    const long long n = ctl->step + kstep;
    const int b = (int)((ctl->cur + kflip) & 1);
    const double4 *u = (const double4 *)I.u[b];
    double4 *hf = (double4 *)I.half;
    const int L = bl.y * 256 + (int)threadIdx.x;
    const int j = L / I.n_r, i = L - j * I.n_r;
    if (j >= I.n_theta || i >= I.n_r - 1) return;
    const double t = (double)n * I.dt;
    const int nt = I.n_theta;
    P4 out;
    if (j >= 1 && j <= nt - 2) {
        out = stage1_at(I, u, i, j, t);
    } else if (!I.m_even) {
        out = zero4();
    } else {
        const int j1 = j == 0 ? 1 : nt - 2, j2 = j == 0 ? 2 : nt - 3;
        out = pole_bc(stage1_at(I, u, i, j1, t), stage1_at(I, u, i, j2, t));
    }
    st_p4(hf + (size_t)j * I.pitch + i, out);
}

__global__ void __launch_bounds__(256) k_two_pass_full(const DevInst *__restrict__ insts, const int2 *__restrict__ blocks,
                                                       const DevCtl *__restrict__ ctl, int kstep, int kflip)
{
    const int2 bl = blocks[blockIdx.x];
    const DevInst &I = insts[bl.x];
    const long long n = ctl->step + kstep;
    const int b = (int)((ctl->cur + kflip) & 1);
    const double4 *u = (const double4 *)I.u[b];
    double4 *un = (double4 *)I.u[b ^ 1];
    const double4 *hf = (const double4 *)I.half;
    const int L = bl.y * 256 + (int)threadIdx.x;
    const int j = L / I.n_r, i = L - j * I.n_r;
    if (j >= I.n_theta) return;
    const double t = (double)n * I.dt + 0.5 * I.dt;
    const int nt = I.n_theta;
    P4 out;
    if (i == 0 || i == I.n_r - 1) {
        out = zero4();
    } else if (j >= 1 && j <= nt - 2) {
        out = stage2_at(I, u, hf, i, j, t);
    } else if (!I.m_even) {
        out = zero4();
    } else {
        const int j1 = j == 0 ? 1 : nt - 2, j2 = j == 0 ? 2 : nt - 3;
        out = pole_bc(stage2_at(I, u, hf, i, j1, t), stage2_at(I, u, hf, i, j2, t));
    }
    st_p4(un + (size_t)j * I.pitch + i, out);
    if (i == I.i_obs && I.extract_every > 0 && (n + 1) % I.extract_every == 0) {
        const long long k = (n + 1) / I.extract_every - 1;
        TK_GLOBAL double *w = gstore_ptr(I.wave) + ((size_t)(k % I.wave_cap) * nt + j) * 2;
        w[0] = out.phi.re;
        w[1] = out.phi.im;
    }
}

__global__ void k_bump(DevCtl *ctl, int n, int flips)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->step += n;
        ctl->cur = (ctl->cur + flips) & 1;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_two_pass(const DevInst *d_inst, const int2 *d_blocks, int n_blocks, const DevCtl *ctl, int kstep,
                           int kflip, hipStream_t s)
{
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_two_pass_half, dim3(n_blocks), dim3(256), 0, s, d_inst, d_blocks, ctl, kstep, kflip);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_two_pass_full, dim3(n_blocks), dim3(256), 0, s, d_inst, d_blocks, ctl, kstep, kflip);
    return hipGetLastError();
}

hipError_t launch_bump(DevCtl *ctl, int n, int flips, hipStream_t s)
{
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, s, ctl, n, flips);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused kernel (FP64, and FP32 with compensated time accumulation).
//
// One wavefront per work item: 64 lanes hold r* columns i0-1 .. i0+62 and
// write the 62 columns i0 .. i0+61; the wave marches over the theta rows of
// its chunk.  At row r it reads u^n row r+1 once (coalesced, prefetched one
// or three rows ahead), takes the neighbour column u^n_{i+1} by a DPP lane
// shift, forms the half-step value at (i+1/2, r) (Eq. (3)), takes
// u^{n+1/2}_{i-1/2} by another shift and forms u^{n+1} at row r-1
// (Eq. (4)).  The half-step array never leaves registers; u^n is read once
// and u^{n+1} written once.  Rolling rows live in three register slots
// indexed by row mod 3 (every index is a compile-time constant inside each
// unrolled phase).  The lane's radial factors (node and half node) are kept
// for the whole march, in registers in FP64 and in LDS in FP32; the angular
// ones are uniform per row.  The two-step kernels (k_fused2 on whole strips,
// k_fused2c on chunks of rows) run a second march three rows behind the
// first on the u^{n+1} rows it leaves in registers; the tiled kernel
// (k_tiled) stages short tiles in LDS instead of marching.  All of them
// compute every point with the same row functions, so their results agree
// bit for bit.
//
// FP32-compensated form: each value is stored as f (FP32) + c (bf16 Kahan
// term).  The stencil runs in FP32 on f; Eq. (4)'s time update is added to
// (f, c) with an exact two-sum, so the accumulated value keeps about 32 bits;
// where the particle source is non-zero its increment is added in FP64.
// ---------------------------------------------------------------------------

namespace {

// Arithmetic / storage policy, prefetch depth (u^n rows in flight per wave:
// 1 or 3), non-temporal stores, and the occupancy the register allocator
// must reach (waves per SIMD; 1 leaves the choice to the compiler, the only
// value compiled: higher targets spill registers, never ran faster, and a
// spill reload can leave the registers of inactive lanes stale, which the
// cross-lane column exchange then reads).
template <int PD, bool NT, int W>
struct PolicyF64 {
    using T = double;
    static constexpr bool kComp = false;
    static constexpr bool kRadRegs = true;  // radial factors in registers (else LDS)
    static constexpr bool kMaskHalo = false;  // lanes off the grid load and compute unmasked
    static constexpr bool kLayer = false;     // instances may end in a hyperboloidal layer
    static constexpr bool kEdge = true;       // a lane may hold a Dirichlet column (see Inner)
    static constexpr int kPD = PD;
    static constexpr bool kNT = NT;
    static constexpr int kWaves = W;
};
// The FP64 form for contexts whose instances may end in a hyperboloidal
// layer (Section 2.3, item 2): the layer's coefficients on the lanes beyond
// rho = R, and the null-infinity column extrapolated inside the march.  The
// kernels run it on the waves that reach the layer only; the others run
// the plain form (Plain), so that their code is the plain kernels' own.
template <int PD, bool NT, int W>
struct PolicyF64L : PolicyF64<PD, NT, W> {
    static constexpr bool kLayer = true;
    using Plain = PolicyF64<3, NT, W>;
};
template <int PD, bool NT, int W>
struct PolicyF32C {
    using T = float;
    static constexpr bool kComp = true;
    static constexpr bool kRadRegs = false;
    static constexpr bool kMaskHalo = true;  // measured faster with them masked
    static constexpr bool kLayer = false;
    static constexpr bool kEdge = true;
    static constexpr int kPD = PD;
    static constexpr bool kNT = NT;
    static constexpr int kWaves = W;
};
// The compensated form's layered counterpart of PolicyF64L: the layer's
// transformation in the differences form's FP32 coefficients, null infinity
// extrapolated from the compensated values in FP64.
template <int PD, bool NT, int W>
struct PolicyF32CL : PolicyF32C<PD, NT, W> {
    static constexpr bool kLayer = true;
    using Plain = PolicyF32C<PD, NT, W>;
};

// A policy's form for waves whose 64 columns all lie strictly inside the
// radial grid (every lane holds a column 1 .. N_r - 2): no lane holds a
// Dirichlet column, so Eq. (4) needs no per-lane zero mask there.  Every
// lane of such a wave computes exactly what the general form computes.
template <class P>
struct Inner : P {
    static constexpr bool kEdge = false;
};

template <typename T>
struct St {  // stored value of a point: f (+ c in the compensated form)
    Q4<T> f, c;
};

// Componentwise choice between two rows (a select of whole structs would
// keep them in memory).
template <typename T>
__device__ __forceinline__ Q4<T> pick(bool c, const Q4<T> &a, const Q4<T> &b)
{
    return Q4<T>{mkc(c ? a.phi.re : b.phi.re, c ? a.phi.im : b.phi.im), mkc(c ? a.pi.re : b.pi.re, c ? a.pi.im : b.pi.im)};
}
template <typename T>
__device__ __forceinline__ St<T> pick(bool c, const St<T> &a, const St<T> &b)
{
    return St<T>{pick(c, a.f, b.f), pick(c, a.c, b.c)};
}

// Neighbour-column exchange inside the wave by DPP wave shifts (a vector
// move, no LDS round trip): shfl_down1 gives lane l the value of lane l+1,
// shfl_up1 that of lane l-1; the lane at the open end gets 0 (bound_ctrl; it
// is a halo lane whose result is never stored).  Every row and bank is
// enabled and bound_ctrl supplies the one lane without a source, so no lane
// keeps an old value: the move takes none, and the destination needs no
// initialisation.
template <int CTRL>
__device__ __forceinline__ int dpp_shift(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
constexpr int kWaveShl1 = 0x130, kWaveShr1 = 0x138;  // wave_shl:1, wave_shr:1
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __builtin_bit_cast(float, dpp_shift<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = dpp_shift<CTRL>((int)(unsigned)b);
    const int hi = dpp_shift<CTRL>((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <class P, typename T>
__device__ __forceinline__ T down1(T v)
{
    return dpp_move<kWaveShl1>(v);
}
template <class P, typename T>
__device__ __forceinline__ T up1(T v)
{
    return dpp_move<kWaveShr1>(v);
}

template <class P, typename T>
__device__ __forceinline__ cx<T> shfl_down1(cx<T> v)
{
    return mkc<T>(down1<P>(v.re), down1<P>(v.im));
}
template <class P, typename T>
__device__ __forceinline__ cx<T> shfl_up1(cx<T> v)
{
    return mkc<T>(up1<P>(v.re), up1<P>(v.im));
}
template <class P, typename T>
__device__ __forceinline__ Q4<T> shfl_down1(const Q4<T> &v)
{
    return Q4<T>{shfl_down1<P>(v.phi), shfl_down1<P>(v.pi)};
}
template <class P, typename T>
__device__ __forceinline__ Q4<T> shfl_up1(const Q4<T> &v)
{
    return Q4<T>{shfl_up1<P>(v.phi), shfl_up1<P>(v.pi)};
}

// A wave-uniform value computed on the vector unit, moved to scalar registers.
__device__ __forceinline__ double uniform(double x)
{
    const unsigned long long b = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ cd uniform(cd v) { return mk(uniform(v.re), uniform(v.im)); }

__device__ __forceinline__ float bf16_to_float(unsigned short b) { return __uint_as_float((unsigned)b << 16); }
__device__ __forceinline__ unsigned short float_to_bf16(float x) { return __builtin_bit_cast(unsigned short, (__bf16)x); }
// x rounded to the nearest bf16 value (the stored precision of the Kahan term)
__device__ __forceinline__ float bf16_round(float x) { return bf16_to_float(float_to_bf16(x)); }

// What one time level of a launch needs besides the lane: the source time
// factors at the start of the step and half a step later, and whether (and
// where in the ring) the step's result is sampled for the waveform.
struct Level {
    cd eh, ef;  // exp(-i m (Omega t + phase0)) at t^n and t^n + dt/2
    bool ext;   // u^{n+1} is a waveform sample
    long long wslot;
};

__device__ __forceinline__ Level make_level(const DevInst &I, long long n)
{
    Level v;
    if (I.src_kind != TK_SRC_NONE) {
        v.eh = uniform(source_phase(I, (double)n * I.dt));
        v.ef = uniform(source_phase(I, (double)n * I.dt + 0.5 * I.dt));
    } else {
        v.eh = v.ef = mk(0, 0);
    }
    v.ext = I.extract_every > 0 && (n + 1) % I.extract_every == 0;
    v.wslot = v.ext ? ((n + 1) / I.extract_every - 1) % I.wave_cap : 0;
    return v;
}

template <class P>
struct Lane {
    using T = typename P::T;
    const DevInst *I;
    // the instance's angular rows, waveform ring and extraction column, read
    // once: the march's stores could alias the descriptor as far as the
    // compiler knows, so reading them through I reloads them on every row
    const Angular *ang;
    const AngularF *angf;
    double *wave;
    int i_obs;
    const void *u, *uc;  // u^n values (and bf16 terms)
    void *un, *unc;      // u^{n+1}
    T *rad;              // this lane's radial factors in LDS: [2 nodes][kRadF/2 pairs] with a stride of 64 pairs
    RadF<T> rf[2];       // or in registers (half node, node)
    int c, p, nt;
    int cl;  // c clamped into the grid: the column this lane reads
    bool hv, icol;
    bool ov;              // this lane's column is one the work item writes
    bool near_h, near_n;  // half node / node lies on the source window
    double gh, gn;        // tabulated A g_r there
    T dt;
    // hyperboloidal layer (kLayer): the lane's map factors in LDS (rho', H,
    // rho'' of the half node at lf[0], lf[64], lf[128], of the node 192
    // further on), whether the half node and the node lie in the layer,
    // whether any lane of the wave has one in it, and whether this lane
    // holds (any lane of the wave holds) the null-infinity column
    const double *lf;
    bool lay_h, lay_n, wlay, scri, wscri;
    // two-step kernels (no layer): this lane's column of the wave's LDS ring
    // [3 slots][half node, node][64 lanes] through which level 1 hands
    // 1/Sigma-hat to level 2
    T *sgr;
};

template <class P>
__device__ __forceinline__ St<typename P::T> load_row(const Lane<P> &L, int row)
{
    using T = typename P::T;
    St<T> v;
    if constexpr (P::kMaskHalo) {
        if (L.cl != L.c) {
            v.f = zero_q4<T>();
            v.c = zero_q4<T>();
            return v;
        }
    }
    const size_t o = (size_t)row * L.p + L.cl;
    if constexpr (!P::kComp) {
        v.f = ld_p4((const double4 *)L.u + o);
    } else {
        const fvec4 a = gload_ptr((const fvec4 *)L.u)[o];
        const hvec4 b = gload_ptr((const hvec4 *)L.uc)[o];
        v.f = Q4<T>{mkc(a.x, a.y), mkc(a.z, a.w)};
        v.c = Q4<T>{mkc(bf16_to_float(b.x), bf16_to_float(b.y)), mkc(bf16_to_float(b.z), bf16_to_float(b.w))};
    }
    return v;
}

// LDS layout of the radial factors: for node k (0 = half node, 1 = node)
// and pair p, lane l reads the two values at ((k kRadF/2 + p) 64 + l) 2.
template <class P>
__device__ __forceinline__ RadF<typename P::T> radf_of(const Lane<P> &L, int k)
{
    using T = typename P::T;
    if constexpr (P::kRadRegs) return L.rf[k];
    typedef T T2 __attribute__((ext_vector_type(2)));
    const T2 *b = (const T2 *)L.rad + k * (kRadF / 2) * 64;
    const T2 v0 = b[0], v1 = b[64], v2 = b[128], v3 = b[192], v4 = b[256];
    return RadF<T>{v0.x, v0.y, v1.x, v1.y, v2.x, v2.y, v3.x, v3.y, v4.x, v4.y};
}

// Uniform angular factors of a row (scalar loads; floats for FP32).
template <class P>
__device__ __forceinline__ AngF<typename P::T> angf_of(const Lane<P> &L, int row)
{
    if constexpr (!P::kComp) {
        const TK_CONST Angular *A = cload_ptr(L.ang) + row;
        return AngF<double>{A->sa, A->sn2, A->kcs, A->V2, A->cot_h};
    } else {
        const TK_CONST AngularF *A = cload_ptr(L.angf) + row;
        return AngF<float>{A->sa, A->sn2, A->kcs, A->V2, A->cot_h};
    }
}

// g_theta of the particle source on a row (0 off its window)
__device__ __forceinline__ double src_theta(const Angular *ang, int row) { return (cload_ptr(ang) + row)->srcg; }

// The bracket's source argument off the source: -0 makes its innermost
// multiply-add a plain multiply.
template <typename T>
__device__ __forceinline__ cx<T> no_source()
{
    return mkc(T(-0.0), T(-0.0));
}

// FP64 form: the source enters the bracket D du / h - S as -F, only on rows
// whose theta factor is non-zero.  The test is on the table entry's bits, a
// wave-uniform scalar comparison, so rows off the window (and instances
// without a source) skip the work; g_r = 0 makes F zero in the other lanes.
__device__ __forceinline__ void add_source(double gq, const Angular *ang, int row, cd e, Q4<double> &br)
{
    const unsigned long long bits = *(const TK_CONST unsigned long long *)&(cload_ptr(ang) + row)->srcg;
    if (bits != 0ull) {
        asm volatile("");  // keeps this a branch: selects would do the work on every row
        const cd F = source_value(gq, __builtin_bit_cast(double, bits), e);
        br.pi = mkc(br.pi.re - F.re, br.pi.im - F.im);
    }
}

template <class P>
__device__ __forceinline__ double value_of(const St<typename P::T> &v, int k)
{
    const typename P::T *f = &v.f.phi.re, *c = &v.c.phi.re;
    return P::kComp ? (double)f[k] + (double)c[k] : (double)f[k];
}

// Waveform sample of an output row (column i_obs) when the level extracts.
template <class P>
__device__ __forceinline__ void sample(const Lane<P> &L, const Level &lv, int row, const St<typename P::T> &v)
{
    if (lv.ext && L.ov && L.c == L.i_obs) {
        TK_GLOBAL double *w = gstore_ptr(L.wave) + ((size_t)lv.wslot * L.nt + row) * 2;
        w[0] = value_of<P>(v, 0);
        w[1] = value_of<P>(v, 1);
    }
}

// Store an output row of u^{n+1} (and sample it).
template <class P>
__device__ __forceinline__ void emit(const Lane<P> &L, const Level &lv, int row, const St<typename P::T> &v)
{
    const size_t o = (size_t)row * L.p + L.c;
    if (L.ov) {
        if constexpr (!P::kComp) {
            const dvec4 x = {v.f.phi.re, v.f.phi.im, v.f.pi.re, v.f.pi.im};
            if (P::kNT)
                __builtin_nontemporal_store(x, gstore_ptr((dvec4 *)L.un) + o);
            else
                gstore_ptr((dvec4 *)L.un)[o] = x;
        } else {
            const fvec4 x = {v.f.phi.re, v.f.phi.im, v.f.pi.re, v.f.pi.im};
            const hvec4 y = {float_to_bf16(v.c.phi.re), float_to_bf16(v.c.phi.im), float_to_bf16(v.c.pi.re),
                             float_to_bf16(v.c.pi.im)};
            if (P::kNT) {
                __builtin_nontemporal_store(x, gstore_ptr((fvec4 *)L.un) + o);
                __builtin_nontemporal_store(y, gstore_ptr((hvec4 *)L.unc) + o);
            } else {
                gstore_ptr((fvec4 *)L.un)[o] = x;
                gstore_ptr((hvec4 *)L.unc)[o] = y;
            }
        }
    }
    sample(L, lv, row, v);
}

// Pole rows (Section 2.2): (4 X1 - X2) / 3 from the two rows next to the
// pole for even m + s, zero for odd m + s.  The parity is selected per component
// (a select between whole structs would keep them in memory).
template <typename T>
__device__ __forceinline__ Q4<T> pole_half(bool even, const Q4<T> &x1, const Q4<T> &x2)
{
    const Q4<T> v = pole_bc(x1, x2);
    const T z = T(0);
    return Q4<T>{mkc(even ? v.phi.re : z, even ? v.phi.im : z), mkc(even ? v.pi.re : z, even ? v.pi.im : z)};
}

// The same on a stored row pair (in double in the compensated form, then
// split back into f + c).
template <class P>
__device__ __forceinline__ St<typename P::T> pole_row(bool even, const St<typename P::T> &x1,
                                                      const St<typename P::T> &x2)
{
    using T = typename P::T;
    St<T> o;
    if constexpr (!P::kComp) {
        o.f = pole_half(even, x1.f, x2.f);
        o.c = zero_q4<T>();
    } else {
        T *of = &o.f.phi.re, *oc = &o.c.phi.re;
        for (int k = 0; k < 4; ++k) {
            const double v = pole_x(value_of<P>(x1, k), value_of<P>(x2, k));
            const T f = (T)v;
            of[k] = even ? f : T(0);
            oc[k] = even ? bf16_round((T)(v - (double)f)) : T(0);
        }
    }
    return o;
}

// A half-step value: one number per component in FP64, a compensated pair
// s + e (both FP32) in the compensated form, so that the rounding of Eq. (3)
// does not reach the differences Eq. (4) takes of it.
template <class P>
using Half = typename std::conditional<P::kComp, St<typename P::T>, Q4<typename P::T>>::type;

// Pole rows of a half-step row: the pair form in double, split into s + e.
template <class P>
__device__ __forceinline__ Half<P> pole_hrow(bool even, const Half<P> &x1, const Half<P> &x2)
{
    using T = typename P::T;
    if constexpr (!P::kComp) {
        return pole_half(even, x1, x2);
    } else {
        St<T> o;
        T *of = &o.f.phi.re, *oc = &o.c.phi.re;
        for (int k = 0; k < 4; ++k) {
            const double v = pole_x(value_of<P>(x1, k), value_of<P>(x2, k));
            const T f = (T)v;
            of[k] = even ? f : T(0);
            oc[k] = even ? (T)(v - (double)f) : T(0);
        }
        return o;
    }
}

template <class P>
__device__ __forceinline__ Half<P> zero_half()
{
    using T = typename P::T;
    if constexpr (!P::kComp) {
        return zero_q4<T>();
    } else {
        return St<T>{zero_q4<T>(), zero_q4<T>()};
    }
}

// exact sum a + b = s + e (two-sum)
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Compensated form: the angular differences of Phi down one column at its
// middle row, from the values x + e of rows j-1 (M), j (Z), j+1 (P): the
// first differences of x and of e separately (a difference of neighbouring
// FP32 values is exact when they are within a factor of two of each other),
// then d2 = d+ - d- and d1 = d+ + d-, each from its two parts.
template <typename T>
struct AngD {
    cx<T> d2, d1;
};
template <typename T>
__device__ __forceinline__ AngD<T> col_diffs(const St<T> &M, const St<T> &Z, const St<T> &P)
{
    AngD<T> a;
    const T *m = &M.f.phi.re, *z = &Z.f.phi.re, *p = &P.f.phi.re;
    const T *mc = &M.c.phi.re, *zc = &Z.c.phi.re, *pc = &P.c.phi.re;
    T *d2 = &a.d2.re, *d1 = &a.d1.re;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const T ep = p[k] - z[k], em = z[k] - m[k];
        const T gp = pc[k] - zc[k], gm = zc[k] - mc[k];
        d2[k] = (ep - em) + (gp - gm);
        d1[k] = (ep + em) + (gp + gm);
    }
    return a;
}

// x1 - x0 for compensated values: (f1 - f0) + (c1 - c0) per component
template <typename T>
__device__ __forceinline__ Q4<T> comp_diff(const St<T> &x1, const St<T> &x0)
{
    return (x1.f - x0.f) + (x1.c - x0.c);
}

// The layer system's coefficients at a point beyond rho = R (Section 2.3,
// item 2), from the plain ones in the fused kernels' factored form.  With the
// map factors rho', H, rho'' of the point (lf[0], lf[64], lf[128]),
// w = rho' b + (1 - b) and v = 1 + H b: the Phi row's speed becomes
// b rho' / w, the Pi row's b rho' / v, d becomes d rho' / (w^2 v), ct becomes
// (ct w + d H + b^2 rho' rho'' - b H b') / (w v), and the angular weights and
// c0 (so the folded c0a) take the factor 1 / (w v).  Near null infinity 1 - b
// is below the rounding of b, so it is formed as -X / Dn with
// X = a^2 Delta sin^2 and Dn = Sh (Sh + rho); then w = num / Dn with
// num = rho' b Dn - X, and one reciprocal r = 1 / (num v) gives
// 1/w = Dn v r, 1/v = num r and 1/(w v) = Dn r.
__device__ __forceinline__ void layer_transform(CoefF<double> &c, const RadF<double> &R, const AngF<double> &A,
                                                const double *lf, double h)
{
    const double rhop = lf[0], H = lf[64], rhopp = lf[128];
    const double b = c.bh * h;
    const double rho = R.rho_h * h;
    const double Sh = c.Sh2 * c.sig;
    const double Dn = Sh * (Sh + rho);
    const double num = fma(rhop * b, Dn, -(R.D2h * A.sa));
    const double v = fma(H, b, 1.0);
    const double r = recip(num * v);  // num v = w v Dn > 0 in the layer
    const double fw = Dn * r;
    const double iw = fw * v, iv = num * r;
    const double bp = R.K * A.sn2 * (c.sig * c.sig) * c.sig;  // b' = K sin^2 W sig
    const double dre = c.dh.re * h, dim = c.dh.im * h;
    const double g = b * b * rhop * rhopp - b * H * bp;
    c.ct = mk(fma(c.ct.re, iv, fma(dre, H, g) * fw), fma(c.ct.im, iv, dim * H * fw));
    const double bh = c.bh * rhop;
    c.bh = bh * iw;
    c.bih = bh * iv;
    const double dd = rhop * iw * fw;
    c.dh = mk(c.dh.re * dd, c.dh.im * dd);
    c.Ap *= fw;
    c.Am *= fw;
    c.c0a = mk(c.c0a.re * fw, c.c0a.im * fw);
}

// The same transformation of the differences form's coefficients (FP32
// arithmetic on the map factors rounded to it; the angular weights A2, A1 and
// c0 take the factor 1 / (w v)).  1 - b is negative and under one per cent of
// rho' b across the layers used here (R >= 10M, a <= 0.99), so w is formed in
// FP32 without cancellation.
__device__ __forceinline__ void layer_transform(CoefD<float> &c, const RadF<float> &R, const AngF<float> &A,
                                                const double *lf, float h)
{
    const float rhop = (float)lf[0], H = (float)lf[64], rhopp = (float)lf[128];
    const float b = c.bh * h;
    const float rho = R.rho_h * h;
    const float Sh = c.Sh2 * c.sig;
    const float Dn = Sh * (Sh + rho);
    const float num = fmaf(rhop * b, Dn, -(R.D2h * A.sa));
    const float v = fmaf(H, b, 1.0f);
    const float r = 1.0f / (num * v);
    const float fw = Dn * r;
    const float iw = fw * v, iv = num * r;
    const float bp = R.K * A.sn2 * (c.sig * c.sig) * c.sig;
    const float dre = c.dh.re * h, dim = c.dh.im * h;
    const float g = b * b * rhop * rhopp - b * H * bp;
    c.ct = mkc(fmaf(c.ct.re, iv, fmaf(dre, H, g) * fw), fmaf(c.ct.im, iv, dim * H * fw));
    const float bh = c.bh * rhop;
    c.bh = bh * iw;
    c.bih = bh * iv;
    const float dd = rhop * iw * fw;
    c.dh = mkc(c.dh.re * dd, c.dh.im * dd);
    c.A2 *= fw;
    c.A1 *= fw;
    c.c0 = mkc(c.c0.re * fw, c.c0.im * fw);
}

// What the stage at a point needs from beyond its own column.  FP64: Phi on
// rows j -+ 1 and the whole row j of the neighbouring column.  Compensated:
// the neighbour's row j (value and term), and the angular differences of Phi
// down both columns.
template <class P, bool COMP = P::kComp>
struct Around;
template <class P>
struct Around<P, false> {
    cx<typename P::T> m;
    Q4<typename P::T> z;
    cx<typename P::T> p;
};
template <class P>
struct Around<P, true> {
    St<typename P::T> z;
    AngD<typename P::T> own, nb;
};

// How the row functions get 1/Sigma-hat at their point (SG), in either
// form: computed (kSigNew), computed and left at sgw for a later level
// (kSigPut), or taken as sgv, the value an earlier level left (kSigGet).
constexpr int kSigNew = 0, kSigPut = 1, kSigGet = 2;

template <class P, int SG>
__device__ __forceinline__ auto coef_at(const Lane<P> &L, int k, int row, typename P::T *sgw, typename P::T sgv)
{
    if constexpr (!P::kComp) {
        if constexpr (SG == kSigGet) return coef_fused_sig(radf_of(L, k), angf_of<P>(L, row), sgv);
        const CoefF<typename P::T> cf = coef_fused(radf_of(L, k), angf_of<P>(L, row));
        if constexpr (SG == kSigPut) *sgw = cf.sig;
        return cf;
    } else {
        if constexpr (SG == kSigGet) return coef_diff_sig(radf_of(L, k), angf_of<P>(L, row), sgv);
        const CoefD<typename P::T> cf = coef_diff(radf_of(L, k), angf_of<P>(L, row));
        if constexpr (SG == kSigPut) *sgw = cf.sig;
        return cf;
    }
}

// The plain FP64 form's W-free coefficients (coef_w_sig), with 1/Sigma-hat
// as coef_at takes it.
template <class P, int SG>
__device__ __forceinline__ CoefW<double> coef_w_at(const Lane<P> &L, int k, int row, double *sgw, double sgv)
{
    const RadF<double> R = radf_of(L, k);
    const AngF<double> A = angf_of<P>(L, row);
    if constexpr (SG == kSigGet) return coef_w_sig(R, A, sgv);
    const double sig = inv_sqrt(fma(-R.D2h, A.sa, R.rho2));
    if constexpr (SG == kSigPut) *sgw = sig;
    return coef_w_sig(R, A, sig);
}

// Eq. (3) at half row r: u^n rows r-1 (UM), r (U0), r+1 (UP) of this column
// and what it needs of the column to the right (nb).
template <class P, int SG = kSigNew>
__device__ __forceinline__ Half<P> half_core(const Lane<P> &L, const Level &lv, const St<typename P::T> &UM,
                                             const St<typename P::T> &U0, const St<typename P::T> &UP,
                                             const Around<P> &nb, int r, typename P::T *sgw = nullptr,
                                             typename P::T sgv = 0)
{
    using T = typename P::T;
    const DevInst &I = *L.I;
    // lanes without a half node (c = n_r - 1 and off the grid) feed only
    // out_row lanes that do not update: computing them unmasked (FP64) or
    // returning zero (FP32C) gives the same stored results
    if constexpr (P::kMaskHalo)
        if (!L.hv) return zero_half<P>();
    const T fac = T(0.5) * L.dt;
    if constexpr (!P::kComp) {
        const Q4<T> du = nb.z - U0.f;
        const Q4<T> bar = mid_from(U0.f, du);
        // a lane outside the layer takes the plain form's value in either
        // form of the wave, so that its bits do not depend on which waves
        // a kernel's work list runs in the layered form
        Q4<T> br = bracket_w(coef_w_at<P, SG>(L, 0, r, sgw, sgv), nb.m + UM.f.phi, nb.p + UP.f.phi, bar.phi, bar.pi, du);
        if constexpr (P::kLayer) {
            if (L.wlay) {
                CoefF<T> cf = coef_at<P, SG>(L, 0, r, sgw, sgv);
                if (L.lay_h) layer_transform(cf, radf_of(L, 0), angf_of<P>(L, r), L.lf, I.h);
                br = pick(L.lay_h,
                          bracket_fused(cf, nb.m + UM.f.phi, nb.p + UP.f.phi, bar.phi, bar.pi, du, no_source<T>()), br);
            }
        }
        add_source(L.gh, L.ang, r, lv.eh, br);
        return lw_update(bar, fac, br);
    } else {
        (void)UM;
        (void)UP;
        const Q4<T> du = comp_diff(nb.z, U0);
        // the average (u_i + u_{i+1}) / 2 = u_i + du / 2 as a pair s + e
        St<T> bar;
        {
            const T *f = &U0.f.phi.re, *c = &U0.c.phi.re, *d = &du.phi.re;
            T *bs = &bar.f.phi.re, *be = &bar.c.phi.re;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                T e;
                two_sum(f[k], T(0.5) * d[k], bs[k], e);
                be[k] = e + c[k];
            }
        }
        CoefD<T> cf = coef_at<P, SG>(L, 0, r, sgw, sgv);
        if constexpr (P::kLayer)
            if (L.wlay && L.lay_h) layer_transform(cf, radf_of(L, 0), angf_of<P>(L, r), L.lf, (T)I.h);
        const Q4<T> br = bracket_diff(cf, nb.own.d2 + nb.nb.d2, nb.own.d1 + nb.nb.d1, bar.f.phi, bar.f.pi, du);
        // u^{n+1/2} = bar - (dt/2) [.] as a pair
        St<T> h;
        {
            const T *bp = &br.phi.re, *bs = &bar.f.phi.re, *be = &bar.c.phi.re;
            T *hs = &h.f.phi.re, *he = &h.c.phi.re;
#pragma unroll
            for (int k = 0; k < 4; ++k) two_sum(bs[k], fma(-fac, bp[k], be[k]), hs[k], he[k]);
        }
        if (L.near_h) {  // FP64 source increment (dt/2) F
            const double gj = src_theta(L.ang, r);
            if (gj != 0.0) {
                const cd F = source_value(L.gh, gj, lv.eh);
                const double f64 = 0.5 * I.dt;
                const double vr = ((double)h.f.pi.re + (double)h.c.pi.re) + f64 * F.re;
                const double vi = ((double)h.f.pi.im + (double)h.c.pi.im) + f64 * F.im;
                h.f.pi = mkc((T)vr, (T)vi);
                h.c.pi = mkc((T)(vr - (double)h.f.pi.re), (T)(vi - (double)h.f.pi.im));
            }
        }
        return h;
    }
}

// The same with the column to the right taken by lane shuffles.
template <class P, int SG = kSigNew>
__device__ __forceinline__ Half<P> half_row(const Lane<P> &L, const Level &lv, const St<typename P::T> &UM,
                                            const St<typename P::T> &U0, const St<typename P::T> &UP, int r,
                                            typename P::T *sgw = nullptr, typename P::T sgv = 0)
{
    Around<P> nb;
    if constexpr (!P::kComp) {
        nb.m = shfl_down1<P>(UM.f.phi);
        nb.z = shfl_down1<P>(U0.f);
        nb.p = shfl_down1<P>(UP.f.phi);
    } else {
        nb.own = col_diffs(UM, U0, UP);
        nb.z.f = shfl_down1<P>(U0.f);
        nb.z.c = shfl_down1<P>(U0.c);
        nb.nb.d2 = shfl_down1<P>(nb.own.d2);
        nb.nb.d1 = shfl_down1<P>(nb.own.d1);
    }
    return half_core<P, SG>(L, lv, UM, U0, UP, nb, r, sgw, sgv);
}

// Eq. (4) at output row o: u^n row o (Uo), half rows o-1 (HM), o (H0), o+1
// (HP) of this column (at c+1/2) and what it needs of the half column at
// c-1/2 (nb).
template <class P, int SG = kSigNew>
__device__ __forceinline__ St<typename P::T> out_core(const Lane<P> &L, const Level &lv, const St<typename P::T> &Uo,
                                                      const Half<P> &HM, const Half<P> &H0, const Half<P> &HP,
                                                      const Around<P> &nb, int o, typename P::T *sgw = nullptr,
                                                      typename P::T sgv = 0)
{
    using T = typename P::T;
    const DevInst &I = *L.I;
    St<T> res;
    res.f = zero_q4<T>();
    res.c = zero_q4<T>();
    if (P::kEdge && !L.icol) return res;
    if constexpr (!P::kComp) {
        const Q4<T> du = H0 - nb.z;
        const Q4<T> til = mid_from(nb.z, du);
        Q4<T> br = bracket_w(coef_w_at<P, SG>(L, 1, o, sgw, sgv), HM.phi + nb.m, HP.phi + nb.p, til.phi, til.pi, du);
        if constexpr (P::kLayer) {
            if (L.wlay) {  // lanes outside the layer keep the plain value (half_core)
                CoefF<T> cf = coef_at<P, SG>(L, 1, o, sgw, sgv);
                if (L.lay_n) layer_transform(cf, radf_of(L, 1), angf_of<P>(L, o), L.lf + 192, I.h);
                br = pick(L.lay_n, bracket_fused(cf, HM.phi + nb.m, HP.phi + nb.p, til.phi, til.pi, du, no_source<T>()),
                          br);
            }
        }
        add_source(L.gn, L.ang, o, lv.ef, br);
        res.f = lw_update(Uo.f, L.dt, br);
    } else {
        (void)HM;
        (void)HP;
        const Q4<T> du = comp_diff(H0, nb.z);
        // the averaged fields enter S only through ct and c0: one FP32 value each
        const Q4<T> til = mid_from(nb.z.f, du);
        CoefD<T> cf = coef_at<P, SG>(L, 1, o, sgw, sgv);
        if constexpr (P::kLayer)
            if (L.wlay && L.lay_n) layer_transform(cf, radf_of(L, 1), angf_of<P>(L, o), L.lf + 192, (T)I.h);
        const Q4<T> br = bracket_diff(cf, nb.own.d2 + nb.nb.d2, nb.own.d1 + nb.nb.d1, til.phi, til.pi, du);
        const T *bp = &br.phi.re, *fp = &Uo.f.phi.re, *cp = &Uo.c.phi.re;
        T *rf = &res.f.phi.re, *rc = &res.c.phi.re;
        const double gj = L.near_n ? src_theta(L.ang, o) : 0.0;
        if (gj != 0.0) {
            // FP64 accumulation where the source injects: u + c - dt [.] + dt F
            const cd F = source_value(L.gn, gj, lv.ef);
            const double add[4] = {0.0, 0.0, I.dt * F.re, I.dt * F.im};
            for (int k = 0; k < 4; ++k) {
                const double v = ((double)fp[k] + (double)cp[k]) + (double)(-L.dt * bp[k]) + add[k];
                rf[k] = (T)v;
                rc[k] = (T)(v - (double)rf[k]);
            }
        } else {
            for (int k = 0; k < 4; ++k) two_sum(fp[k], fma(-L.dt, bp[k], cp[k]), rf[k], rc[k]);
        }
        // the Kahan term is kept at its stored precision from here on, so
        // that a value used on chip equals the value a later step reloads
        for (int k = 0; k < 4; ++k) rc[k] = bf16_round(rc[k]);
    }
    return res;
}

// The same with the half column at c-1/2 taken by lane shuffles.
template <class P, int SG = kSigNew>
__device__ __forceinline__ St<typename P::T> out_row(const Lane<P> &L, const Level &lv, const St<typename P::T> &Uo,
                                                     const Half<P> &HM, const Half<P> &H0, const Half<P> &HP, int o,
                                                     typename P::T *sgw = nullptr, typename P::T sgv = 0)
{
    Around<P> nb;
    if constexpr (!P::kComp) {
        nb.m = shfl_up1<P>(HM.phi);
        nb.z = shfl_up1<P>(H0);
        nb.p = shfl_up1<P>(HP.phi);
    } else {
        nb.own = col_diffs(HM, H0, HP);
        nb.z.f = shfl_up1<P>(H0.f);
        nb.z.c = shfl_up1<P>(H0.c);
        nb.nb.d2 = shfl_up1<P>(nb.own.d2);
        nb.nb.d1 = shfl_up1<P>(nb.own.d1);
    }
    St<typename P::T> v = out_core<P, SG>(L, lv, Uo, HM, H0, HP, nb, o, sgw, sgv);
    if constexpr (P::kLayer) {
        if (L.wscri) {
            // null infinity (Section 2.3, item 2): no characteristic enters,
            // the last node takes the linear extrapolation 2 u_{N-2} - u_{N-3}
            // of the new values of the two columns to its left (in the
            // compensated form in double on f + c, split back into f + c)
            using T = typename P::T;
            if constexpr (!P::kComp) {
                const Q4<T> a = shfl_up1<P>(v.f), b = shfl_up1<P>(a);
                if (L.scri)
                    v.f = Q4<T>{mkc(2.0 * a.phi.re - b.phi.re, 2.0 * a.phi.im - b.phi.im),
                                mkc(2.0 * a.pi.re - b.pi.re, 2.0 * a.pi.im - b.pi.im)};
            } else {
                St<T> a, b;
                a.f = shfl_up1<P>(v.f);
                a.c = shfl_up1<P>(v.c);
                b.f = shfl_up1<P>(a.f);
                b.c = shfl_up1<P>(a.c);
                if (L.scri) {
                    T *of = &v.f.phi.re, *oc = &v.c.phi.re;
                    for (int k = 0; k < 4; ++k) {
                        const double x = 2.0 * value_of<P>(a, k) - value_of<P>(b, k);
                        const T f = (T)x;
                        of[k] = f;
                        oc[k] = bf16_round((T)(x - (double)f));
                    }
                }
            }
        }
    }
    return v;
}

template <class P>
struct Roll {
    using T = typename P::T;
    St<T> U[3];    // u^n(c, row), slot = (row - r_lo) mod 3 (rows r-1, r, r+1 at march row r)
    Half<P> H[3];  // u^{n+1/2}(c+1/2, row), same slots (rows r-2, r-1, r)
    St<T> pre[3];  // prefetched u^n rows (same slots, or slot 0 only at depth 1)
    St<T> keep;    // an output row kept for the pole condition
};

template <class P>
__device__ __forceinline__ St<typename P::T> zero_st()
{
    St<typename P::T> z;
    z.f = zero_q4<typename P::T>();
    z.c = zero_q4<typename P::T>();
    return z;
}

// u^n row r+1 moves from the prefetch ring into the rolling rows, and the
// ring slot is refilled (march row r, slot SR; u_last = last row to read).
template <class P, int SR, class RR>
__device__ __forceinline__ void advance_rows(const Lane<P> &L, RR &R, int r, int u_last)
{
    constexpr int SP = (SR + 1) % 3;
    if constexpr (P::kPD == 3) {
        R.U[SP] = R.pre[SP];  // row r+1; refill its slot with row r+4
        if (r + 4 <= u_last) R.pre[SP] = load_row(L, r + 4);
    } else {
        R.U[SP] = R.pre[0];
        if (r + 2 <= u_last) R.pre[0] = load_row(L, r + 2);
    }
}

// Rows r_lo-1, r_lo into the rolling slots 2 and 0, the next ones into the
// prefetch ring.
template <class P, class RR>
__device__ __forceinline__ void prologue_rows(const Lane<P> &L, RR &R, int r_lo, int u_last)
{
    R.U[2] = load_row(L, r_lo - 1);
    R.U[0] = load_row(L, r_lo);
    if constexpr (P::kPD == 3) {
        R.pre[1] = load_row(L, r_lo + 1);
        if (r_lo + 2 <= u_last) R.pre[2] = load_row(L, r_lo + 2);
        if (r_lo + 3 <= u_last) R.pre[0] = load_row(L, r_lo + 3);
    } else {
        R.pre[0] = load_row(L, r_lo + 1);
    }
}

// One march iteration at half row r (slot SR = (r - r_lo) mod 3).  With
// POLES false the pole and epilogue bookkeeping is compiled out (the
// steady-state rows in the middle of a chunk).
template <class P, int SR, bool POLES>
__device__ __forceinline__ void march(const Lane<P> &L, const Level &lv, Roll<P> &R, int r, int out_lo, int out_hi,
                                      int u_last, bool north)
{
    using T = typename P::T;
    constexpr int SM = (SR + 2) % 3;  // row r-1
    constexpr int SP = (SR + 1) % 3;  // row r+1 (U) / row r-2 (H)
    const int nt = L.nt;
    const bool even = L.I->m_even;
    advance_rows<P, SR>(L, R, r, u_last);
    R.H[SR] = half_row(L, lv, R.U[SM], R.U[SR], R.U[SP], r);
    if (POLES && north && r == 2) R.H[SP] = pole_hrow<P>(even, R.H[SM], R.H[SR]);  // half row 0
    const int o = r - 1;
    if (!POLES || (o >= out_lo && o <= out_hi)) {
        const St<T> v = out_row(L, lv, R.U[SM], R.H[SP], R.H[SM], R.H[SR], o);
        emit(L, lv, o, v);
        if (POLES) {
            if (north && o == 1) R.keep = v;
            if (north && o == 2) emit(L, lv, 0, pole_row<P>(even, R.keep, v));
            if (o == nt - 3) R.keep = v;
        }
    }
}

// South pole after the last march iteration r = nt-2 (slot SR = (nt-2-r_lo) mod 3).
template <class P, int SR>
__device__ __forceinline__ void south(const Lane<P> &L, const Level &lv, Roll<P> &R)
{
    using T = typename P::T;
    constexpr int SM = (SR + 2) % 3;  // row nt-3
    constexpr int SP = (SR + 1) % 3;  // row nt-1 (free slot)
    const int nt = L.nt;
    const bool even = L.I->m_even;
    R.H[SP] = pole_hrow<P>(even, R.H[SR], R.H[SM]);  // half row nt-1
    const St<T> v = out_row(L, lv, R.U[SR], R.H[SM], R.H[SR], R.H[SP], nt - 2);
    emit(L, lv, nt - 2, v);
    emit(L, lv, nt - 1, pole_row<P>(even, v, R.keep));
}

// Two time levels in one pass.  Level 1 is the march above without stores;
// level 2 runs three rows behind it on the u^{n+1} rows level 1 leaves in
// registers and writes u^{n+2}.  Slots are (row - 1) mod 3 for every ring.
template <class P>
struct Roll2 {
    using T = typename P::T;
    St<T> U[3], pre[3];  // u^n rows and the prefetch ring
    Half<P> H[3];        // u^{n+1/2} half rows
    St<T> V[3];          // u^{n+1} rows (level-1 output)
    Half<P> G[3];        // u^{n+3/2} half rows
    St<T> keep;          // a u^{n+2} row kept for a pole
};


// Iteration r (1 <= r <= nt+2, slot S = (r - 1) mod 3).  Level 1 takes
// u^n row r+1 and forms half row r and u^{n+1} row r-1.  Level 2, three rows
// behind, forms half row r-3 of the next step and u^{n+2} row r-4 from
// u^{n+1} rows made in earlier iterations only, so the two levels are
// independent inside an iteration (the new u^{n+1} row enters the ring at
// its end, into the slot level 2 has just finished with).  The pole rows of
// both levels come from the rows next to them as in the one-step march.
// With EDGE false (rows 7 .. nt-2) the pole and end bookkeeping is compiled
// out.  Each ring slot is written from one place only, the rows that feed a
// pole being picked by value: two pole updates of different slots under
// different conditions would otherwise be merged by the compiler into one
// store through a selected address, which keeps the rings in memory.
template <class P, int S, bool EDGE>
__device__ __forceinline__ void march2(const Lane<P> &L, const Level &l1, const Level &l2, Roll2<P> &R, int r)
{
    constexpr int SM = (S + 2) % 3;  // rows r-1 and r-4
    constexpr int SP = (S + 1) % 3;  // rows r+1 and r-2 (and r-5)
    const int nt = L.nt;
    const bool even = L.I->m_even;
    // Level 2 needs Sigma-hat at half row r-3 and node row r-4, the points
    // level 1 took in iteration r-3, which left 1/Sigma-hat in ring slot S;
    // read before level 1 refills the slot.  Where level 2 forms a row here,
    // level 1 formed the same row there (rows 1 .. nt-2 of both kinds).
    using T = typename P::T;
    constexpr bool kShare = !P::kLayer;
    constexpr int SG1 = kShare ? kSigPut : kSigNew, SG2 = kShare ? kSigGet : kSigNew;
    T *const sgh = kShare ? L.sgr + (2 * S) * 64 : nullptr;
    T *const sgn = kShare ? L.sgr + (2 * S + 1) * 64 : nullptr;
    const T sg2h = kShare ? *sgh : T(0), sg2n = kShare ? *sgn : T(0);
    // level 1: half rows r-2 (SP), r-1 (SM), r (S); u^n rows r-1 (SM), r (S), r+1 (SP)
    if (!EDGE || r <= nt - 2) {
        advance_rows<P, S>(L, R, r, nt - 1);
        R.H[S] = half_row<P, SG1>(L, l1, R.U[SM], R.U[S], R.U[SP], r, sgh);
    } else {  // r = nt-1: half row nt-1 from nt-2 (SM), nt-3 (SP); unused after that
        R.H[S] = pole_hrow<P>(even, R.H[SM], R.H[SP]);
    }
    if (EDGE && r == 2) R.H[SP] = pole_hrow<P>(even, R.H[SM], R.H[S]);  // half row 0 from 1 (SM), 2 (S)
    const bool v_new = !EDGE || (r >= 2 && r <= nt - 1);              // u^{n+1} row r-1 this iteration
    St<typename P::T> vn;
    if (v_new) {
        vn = out_row<P, SG1>(L, l1, R.U[SM], R.H[SP], R.H[SM], R.H[S], r - 1, sgn);
        sample(L, l1, r - 1, vn);
    }
    // level 2: u^{n+1} rows r-4 (SM), r-3 (S), r-2 (SP); its half rows r-5 (SP), r-4 (SM), r-3 (S)
    if (!EDGE || (r >= 4 && r <= nt + 1))
        R.G[S] = half_row<P, SG2>(L, l2, R.V[SM], R.V[S], R.V[SP], r - 3, nullptr, sg2h);
    else if (r == nt + 2)  // half row nt-1 from nt-2 (SM), nt-3 (SP)
        R.G[S] = pole_hrow<P>(even, R.G[SM], R.G[SP]);
    if (EDGE && r == 5) R.G[SP] = pole_hrow<P>(even, R.G[SM], R.G[S]);  // half row 0 from 1 (SM), 2 (S)
    if (!EDGE || (r >= 5 && r <= nt + 2)) {                          // u^{n+2} row o = r-4
        const int o = r - 4;
        const St<typename P::T> v = out_row<P, SG2>(L, l2, R.V[SM], R.G[SP], R.G[SM], R.G[S], o, nullptr, sg2n);
        emit(L, l2, o, v);
        if (EDGE) {
            const bool pn = o == 2, ps = o == nt - 2;  // row 0 from rows 1, 2; row nt-1 from nt-2, nt-3
            if (pn || ps) emit(L, l2, pn ? 0 : nt - 1, pole_row<P>(even, pick(pn, R.keep, v), pick(pn, v, R.keep)));
            if (o == 1 || o == nt - 3) R.keep = v;
        }
    }
    // the new u^{n+1} rows enter the ring where level 2 is done
    if (v_new) R.V[SM] = vn;  // row r-1 replaces row r-4
    if (EDGE && r == 3) {     // row 0 (slot S) from rows 1 (SP) and 2 (SM)
        R.V[S] = pole_row<P>(even, R.V[SP], R.V[SM]);
        sample(L, l1, 0, R.V[S]);
    }
    if (EDGE && r == nt) {  // row nt-1 (slot SM, row nt-4 no longer needed) from nt-2 (SP) and nt-3 (S)
        R.V[SM] = pole_row<P>(even, R.V[SP], R.V[S]);
        sample(L, l1, nt - 1, R.V[SM]);
    }
}

// Rows a chunk [j0, j1) of the two-step kernel works on.  It writes u^{n+2}
// rows [j0, j1); level 2 needs the u^{n+1} rows j0-2 .. j1+1 and level 1
// recomputes them, from the half rows j0-3 .. j1+2 and the u^n rows
// j0-4 .. j1+3.  A chunk that holds a pole runs the pole bookkeeping of the
// whole-strip march; the others keep four rows from either pole, so that
// they never need a pole row.  Iteration r forms level 1's half row r and
// u^{n+1} row r-1, and level 2's half row r-3 and u^{n+2} row r-4.
struct Chunk2 {
    int nt;
    bool north, south;
    int r_lo, r_hi;  // iterations
    int h1_hi;       // last level-1 half row from the stencil
    int v_lo, v_hi;  // level-1 rows (u^{n+1}) from the stencil
    int g_lo, g_hi;  // level-2 half rows from the stencil
    int o_lo, o_hi;  // level-2 rows (u^{n+2}) written from the stencil
};

__device__ __forceinline__ Chunk2 chunk2_of(int nt, int j0, int j1)
{
    Chunk2 B;
    B.nt = nt;
    B.north = j0 == 0;
    B.south = j1 == nt;
    B.r_lo = B.north ? 1 : j0 - 3;
    B.h1_hi = B.south ? nt - 2 : j1 + 2;
    B.v_lo = B.north ? 1 : j0 - 2;
    B.v_hi = B.south ? nt - 2 : j1 + 1;
    B.g_lo = B.north ? 1 : j0 - 1;
    B.g_hi = B.south ? nt - 2 : j1;
    B.o_lo = B.north ? 1 : j0;
    B.o_hi = B.south ? nt - 2 : j1 - 1;
    B.r_hi = B.o_hi + 4;
    return B;
}

// One iteration of the two-step march on a chunk (slot S = (r - r_lo) mod
// 3); the whole-strip march2 with the chunk's bounds.  With EDGE false (all
// bounds inside, no pole event) the checks are compiled out.  u^{n+1} rows
// are sampled for the waveform only on the chunk's own rows, so that halo
// rows computed by two chunks are written once.
template <class P, int S, bool EDGE>
__device__ __forceinline__ void march2c(const Lane<P> &L, const Level &l1, const Level &l2, Roll2<P> &R, int r,
                                        const Chunk2 &B)
{
    constexpr int SM = (S + 2) % 3;
    constexpr int SP = (S + 1) % 3;
    const int nt = B.nt;
    const bool even = L.I->m_even;
    // level 1's 1/Sigma-hat for level 2 as in march2: the chunk's bounds keep
    // every row level 2 forms among the rows level 1 formed three
    // iterations earlier (g_lo..g_hi within r_lo..h1_hi, o_lo..o_hi within
    // v_lo..v_hi)
    using T = typename P::T;
    constexpr bool kShare = !P::kLayer;
    constexpr int SG1 = kShare ? kSigPut : kSigNew, SG2 = kShare ? kSigGet : kSigNew;
    T *const sgh = kShare ? L.sgr + (2 * S) * 64 : nullptr;
    T *const sgn = kShare ? L.sgr + (2 * S + 1) * 64 : nullptr;
    const T sg2h = kShare ? *sgh : T(0), sg2n = kShare ? *sgn : T(0);
    if (!EDGE || r <= B.h1_hi) {
        advance_rows<P, S>(L, R, r, B.h1_hi + 1);
        R.H[S] = half_row<P, SG1>(L, l1, R.U[SM], R.U[S], R.U[SP], r, sgh);
    } else if (B.south && r == nt - 1) {
        R.H[S] = pole_hrow<P>(even, R.H[SM], R.H[SP]);
    }
    if (EDGE && B.north && r == 2) R.H[SP] = pole_hrow<P>(even, R.H[SM], R.H[S]);
    const bool v_new = !EDGE || (r - 1 >= B.v_lo && r - 1 <= B.v_hi);
    St<typename P::T> vn;
    if (v_new) {
        vn = out_row<P, SG1>(L, l1, R.U[SM], R.H[SP], R.H[SM], R.H[S], r - 1, sgn);
        if (!EDGE || (r - 1 >= B.o_lo && r - 1 <= B.o_hi)) sample(L, l1, r - 1, vn);
    }
    if (!EDGE || (r - 3 >= B.g_lo && r - 3 <= B.g_hi))
        R.G[S] = half_row<P, SG2>(L, l2, R.V[SM], R.V[S], R.V[SP], r - 3, nullptr, sg2h);
    else if (B.south && r == nt + 2)
        R.G[S] = pole_hrow<P>(even, R.G[SM], R.G[SP]);
    if (EDGE && B.north && r == 5) R.G[SP] = pole_hrow<P>(even, R.G[SM], R.G[S]);
    if (!EDGE || (r - 4 >= B.o_lo && r - 4 <= B.o_hi)) {
        const int o = r - 4;
        const St<typename P::T> v = out_row<P, SG2>(L, l2, R.V[SM], R.G[SP], R.G[SM], R.G[S], o, nullptr, sg2n);
        emit(L, l2, o, v);
        if (EDGE) {
            const bool pn = B.north && o == 2, ps = B.south && o == nt - 2;
            if (pn || ps) emit(L, l2, pn ? 0 : nt - 1, pole_row<P>(even, pick(pn, R.keep, v), pick(pn, v, R.keep)));
            if ((B.north && o == 1) || (B.south && o == nt - 3)) R.keep = v;
        }
    }
    if (v_new) R.V[SM] = vn;
    if (EDGE && B.north && r == 3) {
        R.V[S] = pole_row<P>(even, R.V[SP], R.V[SM]);
        sample(L, l1, 0, R.V[S]);
    }
    if (EDGE && B.south && r == nt) {
        R.V[SM] = pole_row<P>(even, R.V[SP], R.V[S]);
        sample(L, l1, nt - 1, R.V[SM]);
    }
}

// Lane set-up shared by the fused kernels: lane `lane` holds r* column
// i0 - halo + lane and the work item writes lanes halo .. halo+cols-1; the
// lane's radial factors (half node, node) go to its LDS slots.
template <class P>
__device__ __forceinline__ void init_lane(Lane<P> &L, const DevInst &I, const WorkItem &it, int lane, int halo,
                                          int cols, int buf, typename P::T *rad, bool load_rad = true,
                                          double *lay = nullptr)
{
    using T = typename P::T;
    L.I = &I;
    L.ang = I.ang;
    L.angf = I.angf;
    L.wave = I.wave;
    L.i_obs = I.i_obs;
    L.u = I.u[buf];
    L.uc = I.c[buf];
    L.un = I.u[buf ^ 1];
    L.unc = I.c[buf ^ 1];
    L.p = I.pitch;
    L.nt = I.n_theta;
    const int nr = I.n_r;
    L.c = it.i0 - halo + lane;
    // a lane off the grid reads the nearest column (or zero, P::kMaskHalo):
    // what it computes reaches only results that are never stored (halo
    // lanes, and the boundary columns, which out_row sets to zero), so lanes
    // can load and compute without masks
    L.cl = L.c < 0 ? 0 : (L.c >= nr ? nr - 1 : L.c);
    L.hv = L.c >= 0 && L.c <= nr - 2;
    L.icol = L.c >= 1 && L.c <= nr - 2;
    L.ov = lane >= halo && lane < halo + cols && L.c < nr;
    L.dt = (T)I.dt;
    L.rad = rad;
    L.sgr = nullptr;
    if (!load_rad) return;  // the radial factors come from another wave (tiled kernel)
    const Radial Rh = load_entry(gload_ptr(I.rad) + (L.hv ? 2 * L.c + 1 : 0));
    const Radial Rn = load_entry(gload_ptr(I.rad) + (L.icol ? 2 * L.c : 0));
    typedef T T2 __attribute__((ext_vector_type(2)));
    T2 *slot = (T2 *)L.rad;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const Radial &R = k == 0 ? Rh : Rn;
        const double v[kRadF] = {R.rho2, R.rho * I.inv_h,   R.ct_re,           R.ct_im0,
                                 R.K,    R.c1_re * I.inv_h, R.c1_im * I.inv_h, 0.5 * R.Dl * I.inv_dth2,
                                 R.c0_re, R.c0_im};
        if constexpr (P::kRadRegs) {
            L.rf[k] = RadF<T>{(T)v[0], (T)v[1], (T)v[2], (T)v[3], (T)v[4],
                              (T)v[5], (T)v[6], (T)v[7], (T)v[8], (T)v[9]};
            continue;
        }
#pragma unroll
        for (int p = 0; p < kRadF / 2; ++p) {
            T2 x;
            x.x = (T)v[2 * p];
            x.y = (T)v[2 * p + 1];
            slot[(k * (kRadF / 2) + p) * 64] = x;
        }
    }
    L.gh = L.hv ? Rh.srcg : 0.0;
    L.gn = L.icol ? Rn.srcg : 0.0;
    L.near_h = L.gh != 0.0;
    L.near_n = L.gn != 0.0;
    if constexpr (P::kLayer) {
        // the map factors go to the wave's LDS area (lay: this lane's
        // column of it), read back by this lane only
        const TK_GLOBAL LayerTab *tab = I.lay_on ? gload_ptr((const LayerTab *)I.lay) : nullptr;
        LayerTab th{0.0, 0.0, 0.0, 0.0}, tn{0.0, 0.0, 0.0, 0.0};
        if (tab != nullptr && L.hv) th = load_entry(tab + (2 * L.c + 1));
        if (tab != nullptr && L.icol) tn = load_entry(tab + 2 * L.c);
        L.lay_h = th.H != 0.0;
        L.lay_n = tn.H != 0.0;
        lay[0] = th.rhop;
        lay[64] = th.H;
        lay[128] = th.rhopp;
        lay[192] = tn.rhop;
        lay[256] = tn.H;
        lay[320] = tn.rhopp;
        L.lf = lay;
        L.scri = tab != nullptr && L.c == nr - 1;
        L.wlay = __any(L.lay_h || L.lay_n) != 0;
        L.wscri = __any(L.scri) != 0;
    }
}

// Whether a wave whose lanes hold columns i0 - halo .. i0 - halo + 63 of the
// item's instance reaches its layer: lay_c0 is the first column with a half
// node (so with every later node) beyond rho = R, and the null-infinity
// column lies beyond it.
__device__ __forceinline__ bool touches_layer(const DevInst &I, const WorkItem &it, int halo)
{
    return I.lay_on != 0 && it.i0 - halo + 63 >= I.lay_c0;
}

// Whether every lane of such a wave holds an interior column (1 .. N_r - 2),
// so that the wave can run a policy's Inner form.
__device__ __forceinline__ bool inner_wave(const DevInst &I, const WorkItem &it, int halo)
{
    return it.i0 - halo >= 1 && it.i0 - halo + 63 <= I.n_r - 2;
}

}  // namespace

// One wave's work item of k_fused (the kernel picks the form).
template <class P>
__device__ __forceinline__ void k_fused_wave(const DevInst &I, const WorkItem &it, int lane, int cols, int buf,
                                              typename P::T *rad, double *lay, long long n)
{
    Lane<P> L;
    init_lane(L, I, it, lane, 1, cols, buf, rad, true, lay);
    const Level lv = make_level(I, n);

    const int nt = I.n_theta;
    const int j0 = it.j0, j1 = it.j1;
    const bool north = j0 == 0, southp = j1 == nt;
    const int r_lo = max(1, j0 - 1), r_hi = min(nt - 2, j1);
    const int out_lo = max(1, j0);
    const int out_hi = southp ? nt - 3 : min(nt - 2, j1 - 1);  // row nt-2 is the south epilogue's
    const int u_last = r_hi + 1;

    Roll<P> R;
    prologue_rows(L, R, r_lo, u_last);
    R.keep = zero_st<P>();
    // head: the first three rows, with the north-pole bookkeeping
    int r = r_lo;
    march<P, 0, true>(L, lv, R, r, out_lo, out_hi, u_last, north);
    if (r + 1 <= r_hi) march<P, 1, true>(L, lv, R, r + 1, out_lo, out_hi, u_last, north);
    if (r + 2 <= r_hi) march<P, 2, true>(L, lv, R, r + 2, out_lo, out_hi, u_last, north);
    r += 3;
    // steady state: whole triples strictly before the last row (its output
    // row o = r_hi - 1 may be the one the south pole needs)
    for (; r + 2 < r_hi; r += 3) {
        march<P, 0, false>(L, lv, R, r, out_lo, out_hi, u_last, north);
        march<P, 1, false>(L, lv, R, r + 1, out_lo, out_hi, u_last, north);
        march<P, 2, false>(L, lv, R, r + 2, out_lo, out_hi, u_last, north);
    }
    // tail
    if (r <= r_hi) march<P, 0, true>(L, lv, R, r, out_lo, out_hi, u_last, north);
    if (r + 1 <= r_hi) march<P, 1, true>(L, lv, R, r + 1, out_lo, out_hi, u_last, north);
    if (r + 2 <= r_hi) march<P, 2, true>(L, lv, R, r + 2, out_lo, out_hi, u_last, north);
    if (southp) {
        switch ((nt - 2 - r_lo) % 3) {
        case 0: south<P, 0>(L, lv, R); break;
        case 1: south<P, 1>(L, lv, R); break;
        default: south<P, 2>(L, lv, R); break;
        }
    }
}

// One step.  The wave index within the block is made uniform explicitly so
// that the work item, the instance descriptor and the angular tables are
// read with scalar loads into scalar registers.
template <class P>
__global__ void __launch_bounds__(64 * kFusedWavesPerBlock) __attribute__((amdgpu_waves_per_eu(P::kWaves, 8)))
    k_fused(const DevInst *__restrict__ insts, const WorkItem *__restrict__ work, int n_work, int cols,
            const DevCtl *__restrict__ ctl, int kstep, int kflip)
{
    using T = typename P::T;
    __shared__ T s_rad[kFusedWavesPerBlock][P::kRadRegs ? 2 : 2 * kRadF * 64];
    __shared__ double s_lay[kFusedWavesPerBlock][P::kLayer ? 6 * 64 : 1];
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int w = (int)blockIdx.x * kFusedWavesPerBlock + wv;
    if (w >= n_work) return;  // whole wave leaves together; no block barriers below
    const WorkItem it = work[w];
    const DevInst &I = insts[it.inst];
    const long long n = ctl->step + kstep;
    const int buf = (int)((ctl->cur + kflip) & 1);
    if constexpr (P::kLayer) {
        // a wave whose columns all stay below the layer runs the plain form
        if (!touches_layer(I, it, 1)) {
            k_fused_wave<typename P::Plain>(I, it, lane, cols, buf, &s_rad[wv][2 * lane], nullptr, n);
            return;
        }
    }
    k_fused_wave<P>(I, it, lane, cols, buf, &s_rad[wv][2 * lane], &s_lay[wv][P::kLayer ? lane : 0], n);
}

namespace {

// LDS staging of the tiled kernel: a stored point as one 4-vector (f) or two
// (f, c in the compensated form), a half point as one.
template <typename T>
struct Vec4Of;
template <>
struct Vec4Of<double> {
    using type = dvec4;
};
template <>
struct Vec4Of<float> {
    using type = fvec4;
};

template <class P>
__device__ __forceinline__ void lds_put(typename Vec4Of<typename P::T>::type *s, int idx, const St<typename P::T> &v)
{
    using V = typename Vec4Of<typename P::T>::type;
    constexpr int KV = P::kComp ? 2 : 1;
    s[idx * KV] = V{v.f.phi.re, v.f.phi.im, v.f.pi.re, v.f.pi.im};
    if constexpr (P::kComp) s[idx * KV + 1] = V{v.c.phi.re, v.c.phi.im, v.c.pi.re, v.c.pi.im};
}

template <class P>
__device__ __forceinline__ St<typename P::T> lds_get(const typename Vec4Of<typename P::T>::type *s, int idx)
{
    using T = typename P::T;
    constexpr int KV = P::kComp ? 2 : 1;
    St<T> v;
    const auto a = s[idx * KV];
    v.f = Q4<T>{mkc(a.x, a.y), mkc(a.z, a.w)};
    if constexpr (P::kComp) {
        const auto b = s[idx * KV + 1];
        v.c = Q4<T>{mkc(b.x, b.y), mkc(b.z, b.w)};
    } else {
        v.c = zero_q4<T>();
    }
    return v;
}

// A half-step value in LDS: one 4-vector (FP64), two (the compensated pair).
template <class P>
__device__ __forceinline__ void lds_put_half(typename Vec4Of<typename P::T>::type *s, int idx, const Half<P> &v)
{
    using V = typename Vec4Of<typename P::T>::type;
    if constexpr (!P::kComp) {
        s[idx] = V{v.phi.re, v.phi.im, v.pi.re, v.pi.im};
    } else {
        s[2 * idx] = V{v.f.phi.re, v.f.phi.im, v.f.pi.re, v.f.pi.im};
        s[2 * idx + 1] = V{v.c.phi.re, v.c.phi.im, v.c.pi.re, v.c.pi.im};
    }
}

template <class P>
__device__ __forceinline__ Half<P> lds_get_half(const typename Vec4Of<typename P::T>::type *s, int idx)
{
    using T = typename P::T;
    if constexpr (!P::kComp) {
        const auto a = s[idx];
        return Q4<T>{mkc(a.x, a.y), mkc(a.z, a.w)};
    } else {
        const auto a = s[2 * idx], b = s[2 * idx + 1];
        return St<T>{Q4<T>{mkc(a.x, a.y), mkc(a.z, a.w)}, Q4<T>{mkc(b.x, b.y), mkc(b.z, b.w)}};
    }
}

}  // namespace

// One step on a tile: the output rows [j0, j1) (at most TRC) of a strip of
// kFusedCols columns, by a block of four waves.  The u^n rows j0-2 .. j1+1
// are staged in LDS (one row per wave at a time), the half rows j0-1 .. j1
// are formed in parallel and kept in LDS, then the output rows, and the pole
// rows last.  A lane's neighbour columns are read from LDS instead of being
// shuffled; every point is computed by the same row functions as in the
// marching kernels, so the results are theirs bit for bit.  Many short tiles
// instead of a few long marches: the shape for grids too small to give the
// marching kernels enough waves.  One work item per block, every wave takes
// part in every barrier.
template <class P, int TRC>
__global__ void __launch_bounds__(64 * kFusedWavesPerBlock)
    k_tiled(const DevInst *__restrict__ insts, const WorkItem *__restrict__ work, const DevCtl *__restrict__ ctl,
            int kstep, int kflip)
{
    using T = typename P::T;
    using V = typename Vec4Of<T>::type;
    constexpr int NW = kFusedWavesPerBlock;
    constexpr int KV = P::kComp ? 2 : 1;
    // the block's four waves share one strip: its radial factors are loaded
    // once, by wave 0, and passed on through LDS (FP64: the register copies
    // and the source factors; FP32C: its LDS slots and the source factors)
    __shared__ T s_rad[P::kRadRegs ? 2 : 2 * kRadF * 64];
    __shared__ double s_share[(P::kRadRegs ? 2 * kRadF + 2 : 2) * 64];
    __shared__ V s_u[(TRC + 4) * 64 * KV];  // u^n rows a_lo .. a_hi
    __shared__ V s_h[(TRC + 2) * 64 * KV];  // half rows h_lo .. h_hi
    __shared__ V s_p[4 * 64 * KV];          // output rows 1, 2 and nt-2, nt-3 for the poles
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const WorkItem it = work[blockIdx.x];
    const DevInst &I = insts[it.inst];
    const long long n = ctl->step + kstep;
    Lane<P> L;
    const bool lead = wv == 0;
    init_lane(L, I, it, lane, 1, kFusedCols, (int)((ctl->cur + kflip) & 1), &s_rad[2 * lane], lead);
    constexpr int NF = P::kRadRegs ? 2 * kRadF : 0;  // factor values passed on in s_share
    if (lead) {
        if constexpr (P::kRadRegs) {
            const T *f = &L.rf[0].rho2;
            for (int k = 0; k < kRadF; ++k) s_share[k * 64 + lane] = (double)f[k];
            f = &L.rf[1].rho2;
            for (int k = 0; k < kRadF; ++k) s_share[(kRadF + k) * 64 + lane] = (double)f[k];
        }
        s_share[NF * 64 + lane] = L.gh;
        s_share[(NF + 1) * 64 + lane] = L.gn;
    }
    const Level lv = make_level(I, n);
    const int nt = I.n_theta;
    const bool even = I.m_even;
    const int j0 = it.j0, j1 = it.j1;
    const bool north = j0 == 0, southp = j1 == nt;
    const int a_lo = max(0, j0 - 2), a_hi = min(nt - 1, j1 + 1);  // u^n rows staged
    const int h_lo = max(1, j0 - 1), h_hi = min(nt - 2, j1);      // half rows formed
    const int o_lo = max(1, j0), o_hi = min(nt - 2, j1 - 1);      // output rows formed
    // neighbour lanes; the lanes at the two ends read their own values, which
    // only reach halo results that are never stored
    const int lr = lane < 63 ? lane + 1 : lane, ll = lane > 0 ? lane - 1 : lane;

    for (int row = a_lo + wv; row <= a_hi; row += NW) lds_put<P>(s_u, (row - a_lo) * 64 + lane, load_row(L, row));
    __syncthreads();
    if (!lead) {
        if constexpr (P::kRadRegs) {
            T *f = &L.rf[0].rho2;
            for (int k = 0; k < kRadF; ++k) f[k] = (T)s_share[k * 64 + lane];
            f = &L.rf[1].rho2;
            for (int k = 0; k < kRadF; ++k) f[k] = (T)s_share[(kRadF + k) * 64 + lane];
        }
        L.gh = s_share[NF * 64 + lane];
        L.gn = s_share[(NF + 1) * 64 + lane];
        L.near_h = L.gh != 0.0;
        L.near_n = L.gn != 0.0;
    }
    for (int r = h_lo + wv; r <= h_hi; r += NW) {
        const int k = (r - a_lo) * 64;
        const St<T> UM = lds_get<P>(s_u, k - 64 + lane), U0 = lds_get<P>(s_u, k + lane);
        const St<T> UP = lds_get<P>(s_u, k + 64 + lane);
        Around<P> nb;
        if constexpr (!P::kComp) {
            nb.m = lds_get<P>(s_u, k - 64 + lr).f.phi;
            nb.z = lds_get<P>(s_u, k + lr).f;
            nb.p = lds_get<P>(s_u, k + 64 + lr).f.phi;
        } else {
            nb.z = lds_get<P>(s_u, k + lr);
            nb.own = col_diffs(UM, U0, UP);
            nb.nb = col_diffs(lds_get<P>(s_u, k - 64 + lr), nb.z, lds_get<P>(s_u, k + 64 + lr));
        }
        lds_put_half<P>(s_h, (r - h_lo) * 64 + lane, half_core(L, lv, UM, U0, UP, nb, r));
    }
    __syncthreads();
    // half row `row` of lane l, the pole rows from the rows next to them
    auto half_at = [&](int row, int l) -> Half<P> {
        if (row == 0) return pole_hrow<P>(even, lds_get_half<P>(s_h, (1 - h_lo) * 64 + l),
                                          lds_get_half<P>(s_h, (2 - h_lo) * 64 + l));
        if (row == nt - 1) return pole_hrow<P>(even, lds_get_half<P>(s_h, (nt - 2 - h_lo) * 64 + l),
                                               lds_get_half<P>(s_h, (nt - 3 - h_lo) * 64 + l));
        return lds_get_half<P>(s_h, (row - h_lo) * 64 + l);
    };
    for (int o = o_lo + wv; o <= o_hi; o += NW) {
        const St<T> Uo = lds_get<P>(s_u, (o - a_lo) * 64 + lane);
        const Half<P> HM = half_at(o - 1, lane), H0 = half_at(o, lane), HP = half_at(o + 1, lane);
        Around<P> nb;
        if constexpr (!P::kComp) {
            nb.m = half_at(o - 1, ll).phi;
            nb.z = half_at(o, ll);
            nb.p = half_at(o + 1, ll).phi;
        } else {
            nb.z = half_at(o, ll);
            nb.own = col_diffs(HM, H0, HP);
            nb.nb = col_diffs(half_at(o - 1, ll), nb.z, half_at(o + 1, ll));
        }
        const St<T> v = out_core(L, lv, Uo, HM, H0, HP, nb, o);
        emit(L, lv, o, v);
        if (north && o <= 2) lds_put<P>(s_p, (o - 1) * 64 + lane, v);
        if (southp && o >= nt - 3) lds_put<P>(s_p, (2 + (nt - 2 - o)) * 64 + lane, v);
    }
    __syncthreads();
    if (north && wv == 0)
        emit(L, lv, 0, pole_row<P>(even, lds_get<P>(s_p, lane), lds_get<P>(s_p, 64 + lane)));
    if (southp && wv == NW - 1)
        emit(L, lv, nt - 1, pole_row<P>(even, lds_get<P>(s_p, 128 + lane), lds_get<P>(s_p, 192 + lane)));
}

// One wave's work item of k_fused2 (the kernel picks the form).
template <class P>
__device__ __forceinline__ void k_fused2_wave(const DevInst &I, const WorkItem &it, int lane, int cols, int buf,
                                               typename P::T *rad, double *lay, typename P::T *sg, long long n)
{
    Lane<P> L;
    init_lane(L, I, it, lane, 2, cols, buf, rad, true, lay);
    L.sgr = sg;
    const Level l1 = make_level(I, n), l2 = make_level(I, n + 1);
    const int nt = I.n_theta;  // >= 5: the six head iterations all exist

    Roll2<P> R;
    prologue_rows(L, R, 1, nt - 1);
    R.keep = zero_st<P>();
    march2<P, 0, true>(L, l1, l2, R, 1);
    march2<P, 1, true>(L, l1, l2, R, 2);
    march2<P, 2, true>(L, l1, l2, R, 3);
    march2<P, 0, true>(L, l1, l2, R, 4);
    march2<P, 1, true>(L, l1, l2, R, 5);
    march2<P, 2, true>(L, l1, l2, R, 6);
    int r = 7;
    for (; r + 2 <= nt - 2; r += 3) {
        march2<P, 0, false>(L, l1, l2, R, r);
        march2<P, 1, false>(L, l1, l2, R, r + 1);
        march2<P, 2, false>(L, l1, l2, R, r + 2);
    }
    // tail: iterations r .. nt+2 (at most six)
    if (r <= nt + 2) march2<P, 0, true>(L, l1, l2, R, r);
    if (r + 1 <= nt + 2) march2<P, 1, true>(L, l1, l2, R, r + 1);
    if (r + 2 <= nt + 2) march2<P, 2, true>(L, l1, l2, R, r + 2);
    if (r + 3 <= nt + 2) march2<P, 0, true>(L, l1, l2, R, r + 3);
    if (r + 4 <= nt + 2) march2<P, 1, true>(L, l1, l2, R, r + 4);
    if (r + 5 <= nt + 2) march2<P, 2, true>(L, l1, l2, R, r + 5);
}

// Two steps (n -> n+2) in one pass over whole column strips: u^n is read
// and u^{n+2} written once; u^{n+1} exists only in registers (and in the
// waveform ring when sampled).
template <class P>
__global__ void __launch_bounds__(64 * kFusedWavesPerBlock) __attribute__((amdgpu_waves_per_eu(P::kWaves, 8)))
    k_fused2(const DevInst *__restrict__ insts, const WorkItem *__restrict__ work, int n_work,
             const DevCtl *__restrict__ ctl, int kstep, int kflip)
{
    using T = typename P::T;
    __shared__ T s_rad[kFusedWavesPerBlock][P::kRadRegs ? 2 : 2 * kRadF * 64];
    __shared__ T s_sig[kFusedWavesPerBlock][6 * 64];  // Lane::sgr
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int w = (int)blockIdx.x * kFusedWavesPerBlock + wv;
    if (w >= n_work) return;  // whole wave leaves together; no block barriers below
    const WorkItem it = work[w];
    const DevInst &I = insts[it.inst];
    const long long n = ctl->step + kstep;
    const int buf = (int)((ctl->cur + kflip) & 1);
    static_assert(!P::kLayer, "layered contexts march whole strips with k_fused2c");
    if (inner_wave(I, it, 2)) {
        // the form without the Dirichlet mask (only in this kernel: a second
        // body made the chunked kernel's short marches measurably slower)
        k_fused2_wave<Inner<P>>(I, it, lane, kFused2Cols, buf, &s_rad[wv][2 * lane], nullptr, &s_sig[wv][lane], n);
        return;
    }
    k_fused2_wave<P>(I, it, lane, kFused2Cols, buf, &s_rad[wv][2 * lane], nullptr, &s_sig[wv][lane], n);
}

// One wave's work item of k_fused2c (the kernel picks the form).
template <class P>
__device__ __forceinline__ void k_fused2c_wave(const DevInst &I, const WorkItem &it, int lane, int cols, int buf,
                                                typename P::T *rad, double *lay, typename P::T *sg, long long n)
{
    Lane<P> L;
    init_lane(L, I, it, lane, 2, cols, buf, rad, true, lay);
    L.sgr = sg;
    const Level l1 = make_level(I, n), l2 = make_level(I, n + 1);
    const Chunk2 B = chunk2_of(I.n_theta, it.j0, it.j1);
    // every check holds from iteration steady_lo on and through steady_hi
    const int steady_lo = B.north ? 7 : B.r_lo + 7;
    const int steady_hi = B.south ? B.nt - 2 : it.j1;

    Roll2<P> R;
    prologue_rows(L, R, B.r_lo, B.h1_hi + 1);
    R.keep = zero_st<P>();
    int r = B.r_lo;
    for (; r < steady_lo && r <= B.r_hi; r += 3) {
        march2c<P, 0, true>(L, l1, l2, R, r, B);
        if (r + 1 <= B.r_hi) march2c<P, 1, true>(L, l1, l2, R, r + 1, B);
        if (r + 2 <= B.r_hi) march2c<P, 2, true>(L, l1, l2, R, r + 2, B);
    }
    for (; r + 2 <= steady_hi; r += 3) {
        march2c<P, 0, false>(L, l1, l2, R, r, B);
        march2c<P, 1, false>(L, l1, l2, R, r + 1, B);
        march2c<P, 2, false>(L, l1, l2, R, r + 2, B);
    }
    for (; r <= B.r_hi; r += 3) {
        march2c<P, 0, true>(L, l1, l2, R, r, B);
        if (r + 1 <= B.r_hi) march2c<P, 1, true>(L, l1, l2, R, r + 1, B);
        if (r + 2 <= B.r_hi) march2c<P, 2, true>(L, l1, l2, R, r + 2, B);
    }
}

// The two-step kernel on chunks of rows (for workloads whose whole strips
// give too few waves): the same march as k_fused2 over the iterations of
// the chunk, level 1 recomputing the u^{n+1} rows of the halo.  Bitwise the
// results of k_fused2 and k_fused.
template <class P>
__global__ void __launch_bounds__(64 * kFusedWavesPerBlock) __attribute__((amdgpu_waves_per_eu(P::kWaves, 8)))
    k_fused2c(const DevInst *__restrict__ insts, const WorkItem *__restrict__ work, int n_work,
              const DevCtl *__restrict__ ctl, int kstep, int kflip)
{
    using T = typename P::T;
    __shared__ T s_rad[kFusedWavesPerBlock][P::kRadRegs ? 2 : 2 * kRadF * 64];
    __shared__ double s_lay[kFusedWavesPerBlock][P::kLayer ? 6 * 64 : 1];
    __shared__ T s_sig[kFusedWavesPerBlock][6 * 64];  // Lane::sgr
    const int lane = (int)(threadIdx.x & 63);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int w = (int)blockIdx.x * kFusedWavesPerBlock + wv;
    if (w >= n_work) return;  // whole wave leaves together; no block barriers below
    const WorkItem it = work[w];
    const DevInst &I = insts[it.inst];
    const long long n = ctl->step + kstep;
    const int buf = (int)((ctl->cur + kflip) & 1);
    if constexpr (P::kLayer) {
        // a wave whose columns all stay below the layer runs the plain form
        if (!touches_layer(I, it, 2)) {
            k_fused2c_wave<typename P::Plain>(I, it, lane, kFused2Cols, buf, &s_rad[wv][2 * lane], nullptr,
                                              &s_sig[wv][lane], n);
            return;
        }
    }
    k_fused2c_wave<P>(I, it, lane, kFused2Cols, buf, &s_rad[wv][2 * lane], &s_lay[wv][P::kLayer ? lane : 0],
                      &s_sig[wv][lane], n);
}

template <class P>
hipError_t launch_as(const DevInst *d_inst, const WorkItem *d_work, int n_work, int cols, const DevCtl *ctl, int kstep,
                     int kflip, bool two_step, bool chunked, hipStream_t s)
{
    if (n_work <= 0) return hipSuccess;
    const int blocks = (n_work + kFusedWavesPerBlock - 1) / kFusedWavesPerBlock;
    // The compensated form marches whole strips with the chunked kernel's
    // code too (a strip is the chunk [0, n_theta), the same march with the
    // same pole bookkeeping): the whole-strip kernel's unrolled head and tail
    // keep its half-step pairs in more registers than the register file
    // holds for two waves per SIMD.  So does the layered FP64 form: on the
    // waves that reach a layer the whole-strip kernel would form both the
    // plain and the layer's bracket in more registers than that.
    if constexpr (P::kComp || P::kLayer) chunked = chunked || two_step;
    if (two_step && chunked)
        hipLaunchKernelGGL(k_fused2c<P>, dim3(blocks), dim3(64 * kFusedWavesPerBlock), 0, s, d_inst, d_work, n_work,
                           ctl, kstep, kflip);
    else if constexpr (!P::kComp && !P::kLayer) {
        if (two_step)
            hipLaunchKernelGGL(k_fused2<P>, dim3(blocks), dim3(64 * kFusedWavesPerBlock), 0, s, d_inst, d_work,
                               n_work, ctl, kstep, kflip);
        else
            hipLaunchKernelGGL(k_fused<P>, dim3(blocks), dim3(64 * kFusedWavesPerBlock), 0, s, d_inst, d_work,
                               n_work, cols, ctl, kstep, kflip);
    } else
        hipLaunchKernelGGL(k_fused<P>, dim3(blocks), dim3(64 * kFusedWavesPerBlock), 0, s, d_inst, d_work, n_work,
                           cols, ctl, kstep, kflip);
    return hipGetLastError();
}

template <template <int, bool, int> class Pol>
hipError_t launch_variant(const DevInst *d_inst, const WorkItem *d_work, int n_work, int cols, const DevCtl *ctl,
                          int kstep, int kflip, const FusedShape &f, hipStream_t s)
{
#define TK_VARIANT(PD, NT, W)                                                                              \
    if (f.prefetch == PD && f.nt == NT && f.waves == W)                                                    \
        return launch_as<Pol<PD, NT, W>>(d_inst, d_work, n_work, cols, ctl, kstep, kflip, f.two_step, f.chunked, s);
    TK_VARIANT(3, true, 1)
    TK_VARIANT(3, false, 1)
    TK_VARIANT(1, true, 1)
    TK_VARIANT(1, false, 1)
#undef TK_VARIANT
    return hipErrorInvalidValue;
}

namespace {

template <template <int, bool, int> class Pol, int TRC>
hipError_t launch_tiled_as(const DevInst *d_inst, const WorkItem *d_work, int n_work, const DevCtl *ctl, int kstep,
                           int kflip, bool nt, hipStream_t s)
{
    if (n_work <= 0) return hipSuccess;
    if (nt)
        hipLaunchKernelGGL((k_tiled<Pol<1, true, 1>, TRC>), dim3(n_work), dim3(64 * kFusedWavesPerBlock), 0, s, d_inst,
                           d_work, ctl, kstep, kflip);
    else
        hipLaunchKernelGGL((k_tiled<Pol<1, false, 1>, TRC>), dim3(n_work), dim3(64 * kFusedWavesPerBlock), 0, s,
                           d_inst, d_work, ctl, kstep, kflip);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_tiled(bool fp64, const DevInst *d_inst, const WorkItem *d_work, int n_work, int rows,
                        const DevCtl *ctl, int kstep, int kflip, bool nt, hipStream_t s)
{
    // a work item has at most rows + 2 rows (the last chunk absorbs a rest
    // of one or two)
    if (rows == 4)
        return fp64 ? launch_tiled_as<PolicyF64, 6>(d_inst, d_work, n_work, ctl, kstep, kflip, nt, s)
                    : launch_tiled_as<PolicyF32C, 6>(d_inst, d_work, n_work, ctl, kstep, kflip, nt, s);
    if (rows == 8)
        return fp64 ? launch_tiled_as<PolicyF64, 10>(d_inst, d_work, n_work, ctl, kstep, kflip, nt, s)
                    : launch_tiled_as<PolicyF32C, 10>(d_inst, d_work, n_work, ctl, kstep, kflip, nt, s);
    return hipErrorInvalidValue;
}

// The layered form is compiled with one u^n row in flight only: with three,
// the layer's extra coefficient work needs more registers than two waves per
// SIMD leave, and the compiler would spill.
hipError_t launch_layered(const DevInst *d_inst, const WorkItem *d_work, int n_work, int cols, const DevCtl *ctl,
                          int kstep, int kflip, const FusedShape &f, hipStream_t s)
{
    if (f.waves != 1) return hipErrorInvalidValue;
    if (f.nt)
        return launch_as<PolicyF64L<1, true, 1>>(d_inst, d_work, n_work, cols, ctl, kstep, kflip, f.two_step,
                                                 f.chunked, s);
    return launch_as<PolicyF64L<1, false, 1>>(d_inst, d_work, n_work, cols, ctl, kstep, kflip, f.two_step, f.chunked,
                                              s);
}

hipError_t launch_layered_comp(const DevInst *d_inst, const WorkItem *d_work, int n_work, int cols, const DevCtl *ctl,
                               int kstep, int kflip, const FusedShape &f, hipStream_t s)
{
    if (f.waves != 1) return hipErrorInvalidValue;
    if (f.nt)
        return launch_as<PolicyF32CL<1, true, 1>>(d_inst, d_work, n_work, cols, ctl, kstep, kflip, f.two_step,
                                                  f.chunked, s);
    return launch_as<PolicyF32CL<1, false, 1>>(d_inst, d_work, n_work, cols, ctl, kstep, kflip, f.two_step,
                                               f.chunked, s);
}

hipError_t launch_fused(bool fp64, const DevInst *d_inst, const WorkItem *d_work, int n_work, int cols,
                        const DevCtl *ctl, int kstep, int kflip, const FusedShape &f, hipStream_t s, bool layered)
{
    if (fp64 && layered) return launch_layered(d_inst, d_work, n_work, cols, ctl, kstep, kflip, f, s);
    if (layered) return launch_layered_comp(d_inst, d_work, n_work, cols, ctl, kstep, kflip, f, s);
    if (fp64) return launch_variant<PolicyF64>(d_inst, d_work, n_work, cols, ctl, kstep, kflip, f, s);
    return launch_variant<PolicyF32C>(d_inst, d_work, n_work, cols, ctl, kstep, kflip, f, s);
}

}  // namespace tk
