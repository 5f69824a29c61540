// HIP kernels of the Teukolsky m-mode stepper (gfx950).
//
// A step is the two-step Lax-Wendroff scheme of Eqs. (3)-(4) with the pole
// and radial conditions of Section 2.2 applied after each step.  Fields are
// stored per point as (Phi.re, Phi.im, Pi.re, Pi.im) on rows of constant
// theta (r* contiguous), so a wavefront's 64 lanes read 64 consecutive r*
// points: 2 KB per row per access in FP64.
#include <hip/hip_runtime.h>

#include "tk_device.h"
#include "tk_kernels.h"

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
    const Radial &R = I.rad[2 * i + 1];
    const Angular &A = I.ang[j];
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
    const Radial &R = I.rad[2 * i];
    const Angular &A = I.ang[j];
    const Coef c = coef_at(R, A);
    const cd F = R.srcg * A.srcg != 0.0 ? source_value(R.srcg, A.srcg, source_phase(I, t)) : mk(0, 0);
    const P4 un = ld_p4(u + (size_t)j * p + i);
    return lw_point(c, un, phm, til.phi, php, til.pi, h1 - h0, I.dt, I.inv_h, I.inv_dth2, I.inv_2dth, F);
}

__global__ void __launch_bounds__(256) k_two_pass_half(const DevInst *__restrict__ insts, const int2 *__restrict__ blocks,
                                                       const DevCtl *__restrict__ ctl, int kstep)
{
    const int2 bl = blocks[blockIdx.x];
    const DevInst &I = insts[bl.x];
    const long long n = ctl->step + kstep;
    const double4 *u = (const double4 *)I.u[n & 1];
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
                                                       const DevCtl *__restrict__ ctl, int kstep)
{
    const int2 bl = blocks[blockIdx.x];
    const DevInst &I = insts[bl.x];
    const long long n = ctl->step + kstep;
    const double4 *u = (const double4 *)I.u[n & 1];
    double4 *un = (double4 *)I.u[(n + 1) & 1];
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
        double *w = I.wave + ((size_t)(k % I.wave_cap) * nt + j) * 2;
        w[0] = out.phi.re;
        w[1] = out.phi.im;
    }
}

__global__ void k_bump(DevCtl *ctl, int n)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->step += n;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_two_pass(const DevInst *d_inst, const int2 *d_blocks, int n_blocks, const DevCtl *ctl, int kstep,
                           hipStream_t s)
{
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_two_pass_half, dim3(n_blocks), dim3(256), 0, s, d_inst, d_blocks, ctl, kstep);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_two_pass_full, dim3(n_blocks), dim3(256), 0, s, d_inst, d_blocks, ctl, kstep);
    return hipGetLastError();
}

hipError_t launch_bump(DevCtl *ctl, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, s, ctl, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused FP64 kernel.
//
// One wavefront per work item: 64 lanes hold r* columns i0-1 .. i0+62 and
// write the 62 columns i0 .. i0+61; the wave marches over the theta rows of
// its chunk.  At row r it reads u^n row r+1 once (coalesced, 2 KB), takes
// the neighbour column u^n_{i+1} by a lane shuffle, forms the half-step
// value at (i+1/2, r) (Eq. (3)), takes u^{n+1/2}_{i-1/2} by a second
// shuffle and forms u^{n+1} at row r-1 (Eq. (4)).  The half-step array never
// leaves registers; u^n is read once and u^{n+1} written once.  Rolling rows
// live in three register slots indexed by row mod 3 (every index is a
// compile-time constant inside each unrolled phase).
// ---------------------------------------------------------------------------

namespace {


struct Lane64 {
    const DevInst *I;
    const double4 *u;
    double4 *un;
    int c, p, nt;
    bool cin, hv, icol, ov;
    bool near_h, near_n;  // this lane's half node / node lies on the source window
    cd e1, e2;            // source time factors at t^n and t^n + dt/2
    long long n;
    bool ext;         // this step writes a waveform sample
    long long wslot;  // its ring slot
};

struct Roll {
    P4 U[3];  // u^n(c, row), slot = row mod 3 (rows r-1, r, r+1 at march row r)
    P4 H[3];  // u^{n+1/2}(c+1/2, row), slot = row mod 3 (rows r-2, r-1, r)
    P4 pre;   // prefetched u^n row
    P4 keep;  // an output row kept for the pole condition
};

__device__ __forceinline__ P4 load_row(const Lane64 &L, int row)
{
    return L.cin ? ld_p4(L.u + (size_t)row * L.p + L.c) : zero4();
}

__device__ __forceinline__ cd shfl_down1(cd v) { return mk(__shfl_down(v.re, 1), __shfl_down(v.im, 1)); }
__device__ __forceinline__ cd shfl_up1(cd v) { return mk(__shfl_up(v.re, 1), __shfl_up(v.im, 1)); }
__device__ __forceinline__ P4 shfl_down1(const P4 &v) { return P4{shfl_down1(v.phi), shfl_down1(v.pi)}; }
__device__ __forceinline__ P4 shfl_up1(const P4 &v) { return P4{shfl_up1(v.phi), shfl_up1(v.pi)}; }
__device__ __forceinline__ cd avg(cd a, cd b) { return mk((a.re + b.re) * 0.5, (a.im + b.im) * 0.5); }

__device__ __forceinline__ void emit(const Lane64 &L, int row, P4 v)
{
    if (L.ov) st_p4(L.un + (size_t)row * L.p + L.c, v);
    if (L.ext && L.ov && L.c == L.I->i_obs) {
        double *w = L.I->wave + ((size_t)L.wslot * L.nt + row) * 2;
        w[0] = v.phi.re;
        w[1] = v.phi.im;
    }
}

// Eq. (3) at half row r: u^n rows r-1 (UM), r (U0), r+1 (UP) of this column;
// the column to the right comes by lane shuffles.
__device__ __forceinline__ P4 half_row(const Lane64 &L, const Radial &Rh, const P4 &UM, const P4 &U0, const P4 &UP,
                                       int r)
{
    const DevInst &I = *L.I;
    const cd nm = shfl_down1(UM.phi), np = shfl_down1(UP.phi);
    const P4 n0 = shfl_down1(U0);
    if (!L.hv) return zero4();
    const P4 bar = half_sum(n0, U0);
    const Angular &A = I.ang[r];
    const Coef cf = coef_at(Rh, A);
    const cd F = L.near_h ? source_value(Rh.srcg, A.srcg, L.e1) : mk(0, 0);
    return lw_point(cf, bar, avg(nm, UM.phi), bar.phi, avg(np, UP.phi), bar.pi, n0 - U0, 0.5 * I.dt, I.inv_h,
                    I.inv_dth2, I.inv_2dth, F);
}

// Eq. (4) at output row o: half rows o-1 (HM), o (H0), o+1 (HP) of this
// column (at c+1/2); the column at c-1/2 comes by lane shuffles.
__device__ __forceinline__ P4 out_row(const Lane64 &L, const Radial &Rn, const P4 &Uo, const P4 &HM, const P4 &H0,
                                      const P4 &HP, int o)
{
    const DevInst &I = *L.I;
    const cd lm = shfl_up1(HM.phi), lp = shfl_up1(HP.phi);
    const P4 l0 = shfl_up1(H0);
    if (!L.icol) return zero4();
    const P4 til = half_sum(H0, l0);
    const Angular &A = I.ang[o];
    const Coef cf = coef_at(Rn, A);
    const cd F = L.near_n ? source_value(Rn.srcg, A.srcg, L.e2) : mk(0, 0);
    return lw_point(cf, Uo, avg(HM.phi, lm), til.phi, avg(HP.phi, lp), til.pi, H0 - l0, I.dt, I.inv_h, I.inv_dth2,
                    I.inv_2dth, F);
}

// One march iteration at half row r (slot SR = r mod 3).
template <int SR>
__device__ __forceinline__ void march(const Lane64 &L, const Radial &Rh, const Radial &Rn, Roll &R, int r,
                                      int out_lo, int out_hi, int u_last, bool north)
{
    constexpr int SM = (SR + 2) % 3;  // row r-1
    constexpr int SP = (SR + 1) % 3;  // row r+1 (U) / row r-2 (H)
    const DevInst &I = *L.I;
    R.U[SP] = R.pre;
    if (r + 2 <= u_last) R.pre = load_row(L, r + 2);
    R.H[SR] = half_row(L, Rh, R.U[SM], R.U[SR], R.U[SP], r);
    if (north && r == 2) R.H[SP] = I.m_even ? pole_bc(R.H[SM], R.H[SR]) : zero4();  // half row 0
    const int o = r - 1;
    if (o >= out_lo && o <= out_hi) {
        const P4 v = out_row(L, Rn, R.U[SM], R.H[SP], R.H[SM], R.H[SR], o);
        emit(L, o, v);
        if (north && o == 1) R.keep = v;
        if (north && o == 2) emit(L, 0, I.m_even ? pole_bc(R.keep, v) : zero4());
        if (o == I.n_theta - 3) R.keep = v;
    }
}

// South pole after the last march iteration r = nt-2 (slot SR = (nt-2) mod 3).
template <int SR>
__device__ __forceinline__ void south(const Lane64 &L, const Radial &Rn, Roll &R)
{
    constexpr int SM = (SR + 2) % 3;  // row nt-3
    constexpr int SP = (SR + 1) % 3;  // row nt-1 (free slot)
    const DevInst &I = *L.I;
    const int nt = I.n_theta;
    R.H[SP] = I.m_even ? pole_bc(R.H[SR], R.H[SM]) : zero4();  // half row nt-1
    const P4 v = out_row(L, Rn, R.U[SR], R.H[SM], R.H[SR], R.H[SP], nt - 2);
    emit(L, nt - 2, v);
    emit(L, nt - 1, I.m_even ? pole_bc(v, R.keep) : zero4());
}

}  // namespace

__global__ void __launch_bounds__(256) k_fused_fp64(const DevInst *__restrict__ insts, const WorkItem *__restrict__ work,
                                                    int n_work, const DevCtl *__restrict__ ctl, int kstep)
{
    const int lane = (int)(threadIdx.x & 63);
    const int w = (int)blockIdx.x * kFusedWavesPerBlock + (int)(threadIdx.x >> 6);
    if (w >= n_work) return;  // whole wave leaves together
    const WorkItem it = work[w];
    const DevInst &I = insts[it.inst];
    Lane64 L;
    L.I = &I;
    L.n = ctl->step + kstep;
    L.u = (const double4 *)I.u[L.n & 1];
    L.un = (double4 *)I.u[(L.n + 1) & 1];
    L.p = I.pitch;
    L.nt = I.n_theta;
    const int nr = I.n_r, nt = I.n_theta;
    L.c = it.i0 - 1 + lane;
    L.cin = L.c >= 0 && L.c < nr;
    L.hv = L.c >= 0 && L.c <= nr - 2;
    L.icol = L.c >= 1 && L.c <= nr - 2;
    L.ov = lane >= 1 && lane <= kFusedCols && L.c < nr;
    if (I.src_kind == TK_SRC_CIRCULAR_GAUSSIAN) {
        L.e1 = source_phase(I, (double)L.n * I.dt);
        L.e2 = source_phase(I, (double)L.n * I.dt + 0.5 * I.dt);
    } else {
        L.e1 = L.e2 = mk(0, 0);
    }
    L.ext = I.extract_every > 0 && (L.n + 1) % I.extract_every == 0;
    L.wslot = L.ext ? ((L.n + 1) / I.extract_every - 1) % I.wave_cap : 0;

    Radial Rh, Rn;
    if (L.hv) Rh = I.rad[2 * L.c + 1];
    else Rh = I.rad[0];
    if (L.icol) Rn = I.rad[2 * L.c];
    else Rn = I.rad[0];
    L.near_h = L.hv && Rh.srcg != 0.0;
    L.near_n = L.icol && Rn.srcg != 0.0;

    const int j0 = it.j0, j1 = it.j1;
    const bool north = j0 == 0, southp = j1 == nt;
    const int r_lo = max(1, j0 - 1), r_hi = min(nt - 2, j1);
    const int out_lo = max(1, j0), out_hi = min(nt - 3, j1 - 1);  // row nt-2 is the south epilogue's
    const int u_last = r_hi + 1;
    const int out_hi_loop = southp ? out_hi : min(nt - 2, j1 - 1);

    Roll R;
    // prologue: u^n rows r_lo-1 and r_lo, prefetch r_lo+1
    {
        const int a = r_lo - 1, b = r_lo;
        const P4 va = load_row(L, a), vb = load_row(L, b);
        R.pre = load_row(L, b + 1);
        switch (a % 3) {
        case 0: R.U[0] = va; R.U[1] = vb; break;
        case 1: R.U[1] = va; R.U[2] = vb; break;
        default: R.U[2] = va; R.U[0] = vb; break;
        }
    }
    R.keep = zero4();
    for (int r = r_lo; r <= r_hi; ++r) {
        switch (r % 3) {
        case 0: march<0>(L, Rh, Rn, R, r, out_lo, out_hi_loop, u_last, north); break;
        case 1: march<1>(L, Rh, Rn, R, r, out_lo, out_hi_loop, u_last, north); break;
        default: march<2>(L, Rh, Rn, R, r, out_lo, out_hi_loop, u_last, north); break;
        }
    }
    if (southp) {
        switch ((nt - 2) % 3) {
        case 0: south<0>(L, Rn, R); break;
        case 1: south<1>(L, Rn, R); break;
        default: south<2>(L, Rn, R); break;
        }
    }
}

hipError_t launch_fused_fp64(const DevInst *d_inst, const WorkItem *d_work, int n_work, const DevCtl *ctl, int kstep,
                             hipStream_t s)
{
    if (n_work <= 0) return hipSuccess;
    const int blocks = (n_work + kFusedWavesPerBlock - 1) / kFusedWavesPerBlock;
    hipLaunchKernelGGL(k_fused_fp64, dim3(blocks), dim3(64 * kFusedWavesPerBlock), 0, s, d_inst, d_work, n_work, ctl,
                       kstep);
    return hipGetLastError();
}

hipError_t launch_fused_fp32c(const DevInst *, const WorkItem *, int, const DevCtl *, int, hipStream_t)
{
    return hipErrorNotSupported;
}

}  // namespace tk
