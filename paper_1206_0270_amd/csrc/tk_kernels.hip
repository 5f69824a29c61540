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
    const cd F = source_at(I, t, R.rstar, A.theta);
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
    const cd F = source_at(I, t, R.rstar, A.theta);
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

__device__ __forceinline__ P4 shfl_down1(P4 v)
{
    return P4{mk(__shfl_down(v.phi.re, 1), __shfl_down(v.phi.im, 1)),
              mk(__shfl_down(v.pi.re, 1), __shfl_down(v.pi.im, 1))};
}
__device__ __forceinline__ P4 shfl_up1(P4 v)
{
    return P4{mk(__shfl_up(v.phi.re, 1), __shfl_up(v.phi.im, 1)), mk(__shfl_up(v.pi.re, 1), __shfl_up(v.pi.im, 1))};
}

struct Lane64 {
    const DevInst *I;
    const double4 *u;
    double4 *un;
    int c, p, nt;
    bool cin, hv, icol, ov;
    bool near_h, near_n;
    double t1, t2;
    long long n;
    bool ext;         // this step writes a waveform sample
    long long wslot;  // its ring slot
};

struct Roll {
    P4 U[3];   // u^n(c, row)
    P4 B[3];   // (u^n(c+1,row) + u^n(c,row)) / 2
    P4 DU[3];  // u^n(c+1,row) - u^n(c,row)
    P4 HT[3];  // (h(c+1/2,row) + h(c-1/2,row)) / 2
    P4 DH[3];  // h(c+1/2,row) - h(c-1/2,row)
    P4 pre;    // prefetched u^n row
    P4 keep;   // an output row kept for the pole condition
};

__device__ __forceinline__ P4 load_row(const Lane64 &L, int row)
{
    return L.cin ? ld_p4(L.u + (size_t)row * L.p + L.c) : zero4();
}

template <int S>
__device__ __forceinline__ void take_u(Roll &R, P4 own)
{
    const P4 nb = shfl_down1(own);
    R.U[S] = own;
    R.B[S] = half_sum(nb, own);
    R.DU[S] = nb - own;
}

__device__ __forceinline__ void emit(const Lane64 &L, int row, P4 v)
{
    if (L.ov) st_p4(L.un + (size_t)row * L.p + L.c, v);
    if (L.ext && L.ov && L.c == L.I->i_obs) {
        double *w = L.I->wave + ((size_t)L.wslot * L.nt + row) * 2;
        w[0] = v.phi.re;
        w[1] = v.phi.im;
    }
}

// Eq. (4) at output row o with half rows in slots SM (o-1), S0 (o), SP (o+1).
template <int SM, int S0, int SP>
__device__ __forceinline__ P4 out_row(const Lane64 &L, const Radial &Rn, const Roll &R, int o)
{
    const DevInst &I = *L.I;
    if (!L.icol) return zero4();
    const Angular &A = I.ang[o];
    const Coef cf = coef_at(Rn, A);
    const cd F = L.near_n ? source_at(I, L.t2, Rn.rstar, A.theta) : mk(0, 0);
    return lw_point(cf, R.U[S0], R.HT[SM].phi, R.HT[S0].phi, R.HT[SP].phi, R.HT[S0].pi, R.DH[S0], I.dt, I.inv_h,
                    I.inv_dth2, I.inv_2dth, F);
}

// One march iteration at half row r (slot SR = r mod 3).
template <int SR>
__device__ __forceinline__ void march(const Lane64 &L, const Radial &Rh, const Radial &Rn, Roll &R, int r,
                                      int out_lo, int out_hi, int u_last, bool north)
{
    constexpr int SM = (SR + 2) % 3;  // row r-1 (and r+2)
    constexpr int SP = (SR + 1) % 3;  // row r+1 (and r-2)
    const DevInst &I = *L.I;
    // u^n row r+1 (prefetched last iteration), then prefetch row r+2
    take_u<SP>(R, R.pre);
    if (r + 2 <= u_last) R.pre = load_row(L, r + 2);
    // Eq. (3): half step at (c+1/2, r); row r-1 of B sits in slot SM
    P4 h = zero4();
    if (L.hv) {
        const Angular &A = I.ang[r];
        const Coef cf = coef_at(Rh, A);
        const cd F = L.near_h ? source_at(I, L.t1, Rh.rstar, A.theta) : mk(0, 0);
        h = lw_point(cf, R.B[SR], R.B[SM].phi, R.B[SR].phi, R.B[SP].phi, R.B[SR].pi, R.DU[SR], 0.5 * I.dt, I.inv_h,
                     I.inv_dth2, I.inv_2dth, F);
    }
    const P4 hl = shfl_up1(h);
    R.HT[SR] = half_sum(h, hl);
    R.DH[SR] = h - hl;
    if (north && r == 2) {
        // half-step pole row 0 (slot of row r-2 = SP) from rows 1, 2
        R.HT[SP].phi = I.m_even ? mk(pole_x(R.HT[SM].phi.re, R.HT[SR].phi.re), pole_x(R.HT[SM].phi.im, R.HT[SR].phi.im))
                                : mk(0, 0);
    }
    const int o = r - 1;
    if (o >= out_lo && o <= out_hi) {
        // Eq. (4) at row o = r-1: half rows r-2 (SP), r-1 (SM), r (SR); u^n row r-1 (SM)
        const DevInst &II = I;
        P4 v = zero4();
        if (L.icol) {
            const Angular &A = II.ang[o];
            const Coef cf = coef_at(Rn, A);
            const cd F = L.near_n ? source_at(II, L.t2, Rn.rstar, A.theta) : mk(0, 0);
            v = lw_point(cf, R.U[SM], R.HT[SP].phi, R.HT[SM].phi, R.HT[SR].phi, R.HT[SM].pi, R.DH[SM], II.dt, II.inv_h,
                         II.inv_dth2, II.inv_2dth, F);
        }
        emit(L, o, v);
        if (north && o == 1) R.keep = v;
        if (north && o == 2) emit(L, 0, II.m_even ? pole_bc(R.keep, v) : zero4());
        if (o == II.n_theta - 3) R.keep = v;
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
    R.HT[SP].phi = I.m_even ? mk(pole_x(R.HT[SR].phi.re, R.HT[SM].phi.re), pole_x(R.HT[SR].phi.im, R.HT[SM].phi.im))
                            : mk(0, 0);
    const P4 v = out_row<SM, SR, SP>(L, Rn, R, nt - 2);
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
    L.t1 = (double)L.n * I.dt;
    L.t2 = (double)L.n * I.dt + 0.5 * I.dt;
    L.ext = I.extract_every > 0 && (L.n + 1) % I.extract_every == 0;
    L.wslot = L.ext ? ((L.n + 1) / I.extract_every - 1) % I.wave_cap : 0;

    Radial Rh, Rn;
    if (L.hv) Rh = I.rad[2 * L.c + 1];
    else Rh = I.rad[0];
    if (L.icol) Rn = I.rad[2 * L.c];
    else Rn = I.rad[0];
    L.near_h = L.hv && source_near(I, Rh.rstar);
    L.near_n = L.icol && source_near(I, Rn.rstar);

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
        case 0: take_u<0>(R, va); break;
        case 1: take_u<1>(R, va); break;
        default: take_u<2>(R, va); break;
        }
        switch (b % 3) {
        case 0: take_u<0>(R, vb); break;
        case 1: take_u<1>(R, vb); break;
        default: take_u<2>(R, vb); break;
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
