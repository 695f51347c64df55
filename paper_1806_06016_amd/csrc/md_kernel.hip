// PAMD step 3 on gfx950: theta NVT velocity-Verlet steps (Andersen
// collisions) for every replica of a run, in one persistent launch.
//
// Mapping (CDNA wave64):
//   * one replica per 16-lane DPP row, four replicas per wavefront; lane l of a
//     row owns atoms a = 16 s + l (s < NS) and keeps their positions,
//     velocities and forces in VGPRs for all theta steps (HBM is touched once
//     per replica per call);
//   * all-pairs nonbonded forces as 16 x 16 tiles: in tile (I, J) step k lane
//     l pairs atom 16 I + l with atom 16 J + ((l - k) mod 16), read from the
//     neighbour lane with a DPP row rotation folded into the VALU operand;
//     the reaction force returns by the opposite rotation (Newton's third
//     law, every unordered pair evaluated once);
//   * per-(tile, step, lane) pair coefficients (LJ 12 c12, -6 c6 and the
//     Coulomb factor with exclusions / 1-4 scaling folded in) sit in LDS,
//     shared by every replica of the workgroup;
//   * bonded terms: positions are staged in a per-replica LDS slice, each
//     lane evaluates one term per pass and scatters its forces with plain LDS
//     read-modify-writes (terms packed so that no two lanes of a pass touch
//     the same atom in the same role);
//   * persistent workgroups pull groups of four replicas from a device work
//     counter, so the launch needs no host-side knowledge of R.
//
// Functional form (the paper uses AMBER ff94): harmonic bonds and angles,
// Fourier dihedrals with delta in {0, pi} evaluated through Chebyshev
// polynomials of cos(phi), LJ + Coulomb (1/r or eps(r) = 4 r).
#include <type_traits>
#include <utility>

#include "pamd.h"
#include "pamd_internal.h"
#include "philox.h"

namespace pamd {

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// lane l of a 16-lane row receives the value of lane (l - K) mod 16
template <int K>
__device__ __forceinline__ float rowrot(float v)
{
    if constexpr (K == 0) {
        return v;
    } else {
        // bound_ctrl set: no lane of a rotation is out of bounds, and it lets the
        // compiler fold the move into the consuming VALU instruction (DPP operand)
        return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x120 + K,
                                                                  0xF, 0xF, true));
    }
}
template <int K>
__device__ __forceinline__ double rowrot(double v)
{
    if constexpr (K == 0) {
        return v;
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, 0x120 + K, 0xF, 0xF, true);
        const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), 0x120 + K, 0xF, 0xF, true);
        return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    }
}

__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsq_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }   // v_sqrt_f32 (1 ulp)
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Angle in [0, pi] from y = |u x w| >= 0 and x = u.w.  FP32: the octant is
// reduced to t = min / max in [0, 1] and atan(t) = t P(t^2) with an odd
// degree-15 polynomial fitted for this code (iteratively reweighted least
// squares towards minimax over [0, 1]; largest error 1.3e-7 rad evaluated in
// FP32 by Horner's rule), then pi/2 - a above the diagonal and pi - a for
// x < 0.  FP64 keeps the library atan2.
__device__ __forceinline__ float angle_yx(float y, float x)
{
    const float ax = fabsf(x);
    const float mn = fminf(y, ax), mx = fmaxf(y, ax);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float s = t * t;
    float p = -0.004054562654346228f;
    p = p * s + 0.021862942725419998f;
    p = p * s - 0.05591230466961861f;
    p = p * s + 0.09642195701599121f;
    p = p * s - 0.1390862911939621f;
    p = p * s + 0.19946566224098206f;
    p = p * s - 0.33329859375953674f;
    p = p * s + 0.9999993443489075f;
    float a = p * t;
    a = y > ax ? 1.5707963267948966f - a : a;
    return x < 0.0f ? 3.141592653589793f - a : a;
}
__device__ __forceinline__ double angle_yx(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ void sincos_(float a, float* s, float* c) { sincosf(a, s, c); }
__device__ __forceinline__ void sincos_(double a, double* s, double* c) { sincos(a, s, c); }

// LDS ordering between lanes of one wavefront (no workgroup barrier: waves
// of a block run independent work items)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tile schedule, column-major over blocks: for block J, first its diagonal
// block (rotations k = 1..8), then for every rotation k = 0..15 the blocks
// I < J (so the rotated copy of block J is formed once per (J, k)).
__host__ __device__ constexpr int col_base(int J)
{
    int b = 0;
    for (int q = 0; q < J; ++q)
        b += 8 + 16 * q;
    return b;
}

template <typename real, int NS>
struct Regs {
    real x[NS], y[NS], z[NS];
    real vx[NS], vy[NS], vz[NS];
    real fx[NS], fy[NS], fz[NS];
};

// ---------------------------------------------------------------------------
// nonbonded pair step: pair (atom of lane l in block I, atom of lane l-K in block J)
// ---------------------------------------------------------------------------
// pair coefficients of one tile step, loaded one step ahead of their use
template <typename real>
struct Coef {
    real A, nB, C;   // 12 c12 s, -6 c6 s, Coulomb factor (2 k q q s / 4 for eps = 4r; k q q s for 1/r)
};

// ab_lane / c_lane point at this lane's entry of step 0; step st sits a
// constant 16 entries further per step, so every read is an immediate offset
// from one base register
template <int ST, typename real>
__device__ __forceinline__ Coef<real> load_coef(const real* ab_lane, const real* c_lane)
{
    Coef<real> c;
    c.A = ab_lane[ST * 32];
    c.nB = ab_lane[ST * 32 + 1];
    c.C = c_lane[ST * 16];
    return c;
}

// ACC: (fxj, fyj, fzj) is an unrotated accumulator of the partner's reaction
// forces, rotated back once by the caller after all the pair steps that share
// the partner block and rotation; otherwise the reaction goes straight to the
// partner's force by the opposite rotation
template <typename real, int DIEL, int KBACK, bool ENERGY, bool ACC = false>
__device__ __forceinline__ void pair_step(real xi, real yi, real zi, real xjr, real yjr, real zjr,
                                          real& fxi, real& fyi, real& fzi, real& fxj, real& fyj,
                                          real& fzj, const Coef<real>& cf, double& eacc)
{
    // (xjr, yjr, zjr): position of the partner atom, already rotated to this lane
    const real A = cf.A, nB = cf.nB, C = cf.C;
    const real dx = xjr - xi;
    const real dy = yjr - yi;
    const real dz = zjr - zi;
    const real r2 = dx * dx + dy * dy + dz * dz;
    if constexpr (ENERGY) {
        const real ir2 = rcp_(r2);
        const real ir6 = ir2 * ir2 * ir2;
        const real ulj = ir6 * (A * (real)(1.0 / 12.0) * ir6 + nB * (real)(1.0 / 6.0));
        real uc;
        if constexpr (DIEL == 1)
            uc = (real)0.5 * C * ir2;
        else
            uc = C * rsq_(r2);
        eacc += (double)ulj + (double)uc;
    } else {
        real fs;
        if constexpr (DIEL == 1) {
            const real ir2 = rcp_(r2);
            const real ir4 = ir2 * ir2;
            const real ir6 = ir4 * ir2;
            const real t1 = A * ir6 + nB;
            fs = (t1 * ir4 + C) * ir4;
        } else {
            const real ir = rsq_(r2);
            const real ir2 = ir * ir;
            const real ir4 = ir2 * ir2;
            const real ir6 = ir4 * ir2;
            const real t1 = A * ir6 + nB;
            fs = t1 * ir4 * ir4 + C * ir2 * ir;
        }
        // force on i = fs (x_i - x_j) = -fs d ; on j = +fs d
        if constexpr (ACC) {
            fxi = fma_(-fs, dx, fxi);
            fyi = fma_(-fs, dy, fyi);
            fzi = fma_(-fs, dz, fzi);
            fxj = fma_(fs, dx, fxj);
            fyj = fma_(fs, dy, fyj);
            fzj = fma_(fs, dz, fzj);
        } else {
            // returned to the lane that owns j by the opposite rotation
            const real tx = fs * dx, ty = fs * dy, tz = fs * dz;
            fxi -= tx;
            fyi -= ty;
            fzi -= tz;
            fxj += rowrot<KBACK>(tx);
            fyj += rowrot<KBACK>(ty);
            fzj += rowrot<KBACK>(tz);
        }
    }
}

template <typename real, int NS, int DIEL, bool ENERGY>
__device__ __forceinline__ void nonbonded(Regs<real, NS>& r, const real* tab_ab, const real* tab_c, int l16,
                                          double& eacc)
{
    constexpr int NST = tile_steps(NS);
    const real* ab_lane = tab_ab + 2 * l16;
    const real* c_lane = tab_c + l16;
    // software pipeline: the LDS reads of step st + 1 are issued before the
    // arithmetic of step st, so their latency hides behind it
    Coef<real> cur = load_coef<0>(ab_lane, c_lane);
    static_for<0, NS>([&](auto Jc) {
        constexpr int J = decltype(Jc)::value;
        constexpr int base = col_base(J);
        // diagonal block J: rotations 1..8 (rotation 8 pairs each atom twice; the
        // table masks lanes 8..15)
        static_for<1, 9>([&](auto Kc) {
            constexpr int K = decltype(Kc)::value;
            constexpr int st = base + K - 1;
            const Coef<real> nxt = load_coef<(st + 1 < NST ? st + 1 : st)>(ab_lane, c_lane);
            pair_step<real, DIEL, (16 - K) & 15, ENERGY>(r.x[J], r.y[J], r.z[J], rowrot<K>(r.x[J]),
                                                         rowrot<K>(r.y[J]), rowrot<K>(r.z[J]), r.fx[J], r.fy[J],
                                                         r.fz[J], r.fx[J], r.fy[J], r.fz[J], cur, eacc);
            cur = nxt;
            // one pair step per scheduling region: the steps are independent up
            // to the force sums, and an unbounded window hoists the displacement
            // math of many steps into spilled registers
            __builtin_amdgcn_sched_barrier(0);
        });
        // blocks I < J against block J rotated by K: the reactions of the J
        // pair steps that share this rotated copy accumulate unrotated and go
        // back to block J by one opposite rotation
        if constexpr (J > 0) {
            static_for<0, 16>([&](auto Kc) {
                constexpr int K = decltype(Kc)::value;
                const real xr = rowrot<K>(r.x[J]), yr = rowrot<K>(r.y[J]), zr = rowrot<K>(r.z[J]);
                real gx = (real)0, gy = (real)0, gz = (real)0;
                static_for<0, J>([&](auto Ic) {
                    constexpr int I = decltype(Ic)::value;
                    constexpr int st = base + 8 + K * J + I;
                    const Coef<real> nxt = load_coef<(st + 1 < NST ? st + 1 : st)>(ab_lane, c_lane);
                    pair_step<real, DIEL, (16 - K) & 15, ENERGY, true>(r.x[I], r.y[I], r.z[I], xr, yr, zr, r.fx[I],
                                                                       r.fy[I], r.fz[I], gx, gy, gz, cur, eacc);
                    cur = nxt;
                    __builtin_amdgcn_sched_barrier(0);
                });
                if constexpr (!ENERGY) {
                    r.fx[J] += rowrot<(16 - K) & 15>(gx);
                    r.fy[J] += rowrot<(16 - K) & 15>(gy);
                    r.fz[J] += rowrot<(16 - K) & 15>(gz);
                }
            });
        }
    });
}

// ---------------------------------------------------------------------------
// bonded terms on the LDS stage of one replica (pos, frc: [n][3])
// ---------------------------------------------------------------------------
template <typename real>
__device__ __forceinline__ void ld3(const real* p, int a, real* v)
{
    v[0] = p[3 * a];
    v[1] = p[3 * a + 1];
    v[2] = p[3 * a + 2];
}

// Scatter of a bonded-term force into the replica's LDS force stage.  Plain
// read-modify-write (LDS float atomics are far slower): the host packs the
// terms so that, within one pass of 16 lanes, no two lanes name the same atom
// in the same role, and the roles are scattered one after the other.
template <typename real, bool ENERGY>
__device__ __forceinline__ void add3(real* frc, int a, real fx, real fy, real fz)
{
    if constexpr (!ENERGY) {
        frc[3 * a] += fx;
        frc[3 * a + 1] += fy;
        frc[3 * a + 2] += fz;
    }
}

// One lane per centre atom j with up to NO outer atoms (NO = 4: the six
// angles of the outer pairs; NO = 3: the three pairs of outer roles 0..2):
// each bond vector u_a = x_a - x_j is normalised once (e_a), and the force on
// outer atom a of angle (a, j, c) is -k dth (cos theta e_a - e_c) / (|u_a| sin theta);
// the bonds j - a folded into the group add -k_b (|u_a| - r0) e_a; the centre
// takes minus the sum.
template <typename real, bool ENERGY, int NO>
__device__ __forceinline__ void angle_group(const RunDev<real>& d, const real* pos, real* frc, int t, double& eacc)
{
    const int4 ga = d.agrp[2 * t];
    if (ga.x < 0)
        return;
    const int oa[4] = {ga.y, ga.z, ga.w, NO == 4 ? d.agrp[2 * t + 1].x : -1};
    const real* par = d.agpar + kAngPar * t;
    real pj[3];
    ld3(pos, ga.x, pj);
    real e[NO][3], iu[NO], hb[NO];
#pragma unroll
    for (int a = 0; a < NO; ++a) {
        real pa[3];
        ld3(pos, oa[a] >= 0 ? oa[a] : ga.x, pa);
        const real ux = pa[0] - pj[0], uy = pa[1] - pj[1], uz = pa[2] - pj[2];
        const real u2 = ux * ux + uy * uy + uz * uz;
        // absent outer atoms (their angles and bond carry k = 0): a unit vector along x
        iu[a] = oa[a] >= 0 ? rsq_(u2) : (real)1;
        e[a][0] = oa[a] >= 0 ? ux * iu[a] : (real)1;
        e[a][1] = uy * iu[a];
        e[a][2] = uz * iu[a];
        // bond j - a: U = 1/2 k_b (|u_a| - r0)^2, its force on a is -hb e_a
        const real kb = par[12 + 2 * a], dr = u2 * iu[a] - par[13 + 2 * a];
        if constexpr (ENERGY)
            eacc += (double)((real)0.5 * kb * dr * dr);
        hb[a] = kb * dr;
    }
    real S[NO][3];
#pragma unroll
    for (int a = 0; a < NO; ++a)
        S[a][0] = S[a][1] = S[a][2] = (real)0;
    constexpr int NQ = NO * (NO - 1) / 2;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        // outer pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3) at parameter slots 0..5;
        // with three outer atoms (0,1) (0,2) (1,2) at slots 0, 1, 3
        constexpr int A4[6] = {0, 0, 0, 1, 1, 2}, C4[6] = {1, 2, 3, 2, 3, 3};
        constexpr int A3[3] = {0, 0, 1}, C3[3] = {1, 2, 2}, P3[3] = {0, 1, 3};
        const int a = NO == 4 ? A4[q] : A3[q], c = NO == 4 ? C4[q] : C3[q];
        const int ps = NO == 4 ? q : P3[q];
        const real k = par[2 * ps], th0 = par[2 * ps + 1];
        const real cs = e[a][0] * e[c][0] + e[a][1] * e[c][1] + e[a][2] * e[c][2];
        const real cx = e[a][1] * e[c][2] - e[a][2] * e[c][1];
        const real cy = e[a][2] * e[c][0] - e[a][0] * e[c][2];
        const real cz = e[a][0] * e[c][1] - e[a][1] * e[c][0];
        const real sn = sqrt_(cx * cx + cy * cy + cz * cz);
        const real dth = angle_yx(sn, cs) - th0;
        if constexpr (ENERGY) {
            eacc += (double)((real)0.5 * k * dth * dth);
        } else {
            const real g = k * dth * rcp_(sn < (real)1e-8 ? (real)1e-8 : sn);
            S[a][0] += g * (cs * e[a][0] - e[c][0]);
            S[a][1] += g * (cs * e[a][1] - e[c][1]);
            S[a][2] += g * (cs * e[a][2] - e[c][2]);
            S[c][0] += g * (cs * e[c][0] - e[a][0]);
            S[c][1] += g * (cs * e[c][1] - e[a][1]);
            S[c][2] += g * (cs * e[c][2] - e[a][2]);
        }
    }
    if constexpr (!ENERGY) {
        real fj[3] = {(real)0, (real)0, (real)0};
#pragma unroll
        for (int a = 0; a < NO; ++a) {
            const real fx = -fma_(S[a][0], iu[a], hb[a] * e[a][0]);
            const real fy = -fma_(S[a][1], iu[a], hb[a] * e[a][1]);
            const real fz = -fma_(S[a][2], iu[a], hb[a] * e[a][2]);
            fj[0] -= fx;
            fj[1] -= fy;
            fj[2] -= fz;
            if (oa[a] >= 0)
                add3<real, ENERGY>(frc, oa[a], fx, fy, fz);
        }
        add3<real, ENERGY>(frc, ga.x, fj[0], fj[1], fj[2]);
    }
}

// W: lanes per pass (16 in the register-tile layout, 64 in the wide layout);
// the host packs the records in passes of W
template <typename real, bool ENERGY, int W = kRow>
__device__ __forceinline__ void bonded_terms(const RunDev<real>& d, const real* pos, real* frc, int l16, double& eacc)
{
    // bonds no angle group evaluates: U = 1/2 k (r - r0)^2
    for (int t0 = 0; t0 < d.nb; t0 += W) {
        const int t = t0 + l16;
        const int4 ix = d.bidx[t];
        if (ix.x >= 0) {
            const real k = d.bpar[2 * t], r0 = d.bpar[2 * t + 1];
            real pi[3], pj[3];
            ld3(pos, ix.x, pi);
            ld3(pos, ix.y, pj);
            const real dx = pi[0] - pj[0], dy = pi[1] - pj[1], dz = pi[2] - pj[2];
            const real r2 = dx * dx + dy * dy + dz * dz;
            if constexpr (ENERGY) {
                const real dr = sqrt_(r2) - r0;
                eacc += (double)((real)0.5 * k * dr * dr);
            } else {
                // -dU/dx_i = -k (r - r0) d / r = -k (1 - r0 / r) d
                const real g = (r0 == (real)0) ? k : k * ((real)1 - r0 * rsq_(r2));
                add3<real, ENERGY>(frc, ix.x, -g * dx, -g * dy, -g * dz);
                add3<real, ENERGY>(frc, ix.y, g * dx, g * dy, g * dz);
            }
        }
    }
    // angles: U = 1/2 k (theta - theta0)^2, theta = atan2(|e_a x e_c|, e_a . e_c):
    // the groups with four outer atoms (six angles), then those with at most
    // three (three angles)
    for (int t0 = 0; t0 < d.nag6; t0 += W)
        angle_group<real, ENERGY, 4>(d, pos, frc, t0 + l16, eacc);
    for (int t0 = d.nag6; t0 < d.nag; t0 += W)
        angle_group<real, ENERGY, 3>(d, pos, frc, t0 + l16, eacc);
    // dihedrals: U = k (1 + cos(n phi - delta)) = |kc| + kc cos(n phi), kc = k cos(delta), delta in {0, pi}.
    // One lane per group of torsions around one central bond j-k (up to three
    // outer atoms i on the j side, three l on the k side, every (i, l) one
    // torsion): the bond vector b2 is shared, each i contributes its plane
    // normal n1 = b1 x b2 and each l its n2 = b2 x b3 once, and the torsion
    // forces collapse to per-atom sums:  with g_i = -|b2| n1 / |n1|^2,
    // g_l = |b2| n2 / |n2|^2, p_i = b1.b2 / |b2|^2, q_l = b3.b2 / |b2|^2 and
    // D_i = sum_l dU/dphi_il, E_l = sum_i dU/dphi_il:
    //   F_i = -D_i g_i,  F_l = -E_l g_l,
    //   F_j = sum_i (1 + p_i) D_i g_i - sum_l q_l E_l g_l,
    //   F_k = -sum_i p_i D_i g_i + sum_l (1 + q_l) E_l g_l.
    for (int t0 = 0; t0 < d.ng; t0 += W) {
        const int t = t0 + l16;
        const int4 ga = d.dgrp[2 * t], gb = d.dgrp[2 * t + 1];
        if (ga.x >= 0) {
            const int ia[3] = {ga.z, ga.w, gb.x};
            const int la[3] = {gb.y, gb.z, gb.w};
            const real* par = d.dgpar + 45 * t;
            real pj[3], pk[3];
            ld3(pos, ga.x, pj);
            ld3(pos, ga.y, pk);
            const real b2x = pk[0] - pj[0], b2y = pk[1] - pj[1], b2z = pk[2] - pj[2];
            const real b2sq = b2x * b2x + b2y * b2y + b2z * b2z;
            const real lb2 = sqrt_(b2sq);
            const real ib2 = rcp_(b2sq);
            // j side: b1 = x_j - x_i, n1 = b1 x b2, p_i = b1.b2 / |b2|^2
            real n1[3][3], n1sq[3], pi_[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                real pi[3];
                ld3(pos, ia[a] >= 0 ? ia[a] : ga.x, pi);
                const real b1x = pj[0] - pi[0], b1y = pj[1] - pi[1], b1z = pj[2] - pi[2];
                n1[a][0] = b1y * b2z - b1z * b2y;
                n1[a][1] = b1z * b2x - b1x * b2z;
                n1[a][2] = b1x * b2y - b1y * b2x;
                pi_[a] = (b1x * b2x + b1y * b2y + b1z * b2z) * ib2;
                // absent outer atoms (their torsions carry kc = 0) keep every product finite
                const real q2 = n1[a][0] * n1[a][0] + n1[a][1] * n1[a][1] + n1[a][2] * n1[a][2];
                n1sq[a] = ia[a] < 0 ? (real)1 : q2 < (real)1e-30 ? (real)1e-30 : q2;
            }
            // k side, one outer atom l at a time (b3 = x_l - x_k, n2 = b2 x b3,
            // q_l = b3.b2 / |b2|^2): its torsions with every i, then its force
            real Di[3] = {(real)0, (real)0, (real)0};
            real fj[3] = {(real)0, (real)0, (real)0}, fk[3] = {(real)0, (real)0, (real)0};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                real pl[3];
                ld3(pos, la[c] >= 0 ? la[c] : ga.y, pl);
                const real b3x = pl[0] - pk[0], b3y = pl[1] - pk[1], b3z = pl[2] - pk[2];
                const real n2x = b2y * b3z - b2z * b3y;
                const real n2y = b2z * b3x - b2x * b3z;
                const real n2z = b2x * b3y - b2y * b3x;
                const real q2 = n2x * n2x + n2y * n2y + n2z * n2z;
                // absent outer atoms (their torsions carry kc = 0) keep every product finite
                const real n2sq = la[c] < 0 ? (real)1 : q2 < (real)1e-30 ? (real)1e-30 : q2;
                real El = (real)0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const real* tp_ = par + 5 * (3 * a + c);
                    const real kc = tp_[0];
                    const real inn = rsq_(n1sq[a] * n2sq);
                    const real cphi = (n1[a][0] * n2x + n1[a][1] * n2y + n1[a][2] * n2z) * inn;
                    if constexpr (ENERGY) {
                        // Chebyshev: T_n(c) = cos(n phi)
                        const int nmul = (int)tp_[1];
                        real tp = (real)1, tc = cphi;
                        for (int q = 1; q < nmul; ++q) {
                            const real tn = (real)2 * cphi * tc - tp;
                            tp = tc;
                            tc = tn;
                        }
                        eacc += (double)(fabs(kc) + kc * tc);
                    } else {
                        // sin phi = |b2| b1.(b2 x b3) / (|n1| |n2|), and b1.(b2 x b3) = n1.b3
                        const real sphi = lb2 * (n1[a][0] * b3x + n1[a][1] * b3y + n1[a][2] * b3z) * inn;
                        // dU/dphi = -kc n sin(n phi) = -kc n sin(phi) U_{n-1}(cos phi), with
                        // kc n U_{n-1}(c) = c0 + c1 c + c2 c^2 for n <= 3
                        real poly = fma_(fma_(tp_[4], cphi, tp_[3]), cphi, tp_[2]);
                        if (d.dih_general) {
                            // some torsion has n > 3: U_{n-1} by the Chebyshev recurrence
                            const int nmul = (int)tp_[1];
                            real up = (real)0, uc = (real)1;
                            for (int q = 1; q < nmul; ++q) {
                                const real un = (real)2 * cphi * uc - up;
                                up = uc;
                                uc = un;
                            }
                            poly = kc * (real)nmul * uc;
                        }
                        const real dU = -sphi * poly;
                        Di[a] += dU;
                        El += dU;
                    }
                }
                if constexpr (!ENERGY) {
                    // E_l g_l with g_l = |b2| n2 / |n2|^2
                    const real sc = lb2 * rcp_(n2sq) * El;
                    const real gx = sc * n2x, gy = sc * n2y, gz = sc * n2z;
                    const real qc = (b3x * b2x + b3y * b2y + b3z * b2z) * ib2;
                    fj[0] -= qc * gx;
                    fj[1] -= qc * gy;
                    fj[2] -= qc * gz;
                    fk[0] += ((real)1 + qc) * gx;
                    fk[1] += ((real)1 + qc) * gy;
                    fk[2] += ((real)1 + qc) * gz;
                    if (la[c] >= 0)
                        add3<real, ENERGY>(frc, la[c], -gx, -gy, -gz);
                }
            }
            if constexpr (!ENERGY) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    // D_i g_i with g_i = -|b2| n1 / |n1|^2
                    const real sa = -lb2 * rcp_(n1sq[a]) * Di[a];
                    const real gx = sa * n1[a][0], gy = sa * n1[a][1], gz = sa * n1[a][2];
                    const real pa = pi_[a];
                    fj[0] += ((real)1 + pa) * gx;
                    fj[1] += ((real)1 + pa) * gy;
                    fj[2] += ((real)1 + pa) * gz;
                    fk[0] -= pa * gx;
                    fk[1] -= pa * gy;
                    fk[2] -= pa * gz;
                    if (ia[a] >= 0)
                        add3<real, ENERGY>(frc, ia[a], -gx, -gy, -gz);
                }
                add3<real, ENERGY>(frc, ga.x, fj[0], fj[1], fj[2]);
                add3<real, ENERGY>(frc, ga.y, fk[0], fk[1], fk[2]);
            }
        }
    }
}

// TERMS: 1 bonded, 2 nonbonded, 3 both
template <typename real, int NS, int DIEL, bool ENERGY, int TERMS = 3>
__device__ __forceinline__ void evaluate(Regs<real, NS>& r, const RunDev<real>& d, const real* tab_ab,
                                         const real* tab_c, real* pos, real* frc, int l16, double& eacc)
{
    if constexpr (!ENERGY) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            r.fx[s] = (real)0;
            r.fy[s] = (real)0;
            r.fz[s] = (real)0;
        }
    }
    if constexpr ((TERMS & 1) != 0) {
        // stage positions for the bonded terms
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int a = 16 * s + l16;
            if (a < d.n) {
                pos[3 * a] = r.x[s];
                pos[3 * a + 1] = r.y[s];
                pos[3 * a + 2] = r.z[s];
            }
        }
        wave_sync();
        // bonded terms first: their LDS scatter completes while the
        // register-only nonbonded tiles run
        bonded_terms<real, ENERGY>(d, pos, frc, l16, eacc);
    }
    if constexpr ((TERMS & 2) != 0)
        nonbonded<real, NS, DIEL, ENERGY>(r, tab_ab, tab_c, l16, eacc);
    if constexpr (!ENERGY) {
        // materialise the pair-force sums here (otherwise the sums are sunk to
        // their use and every pair's partial force stays live)
#pragma unroll
        for (int s = 0; s < NS; ++s)
            asm volatile("" : "+v"(r.fx[s]), "+v"(r.fy[s]), "+v"(r.fz[s]));
    }
    if constexpr (!ENERGY && (TERMS & 1) != 0) {
        wave_sync();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int a = 16 * s + l16;
            if (a < d.n) {
                r.fx[s] += frc[3 * a];
                r.fy[s] += frc[3 * a + 1];
                r.fz[s] += frc[3 * a + 2];
                frc[3 * a] = (real)0;
                frc[3 * a + 1] = (real)0;
                frc[3 * a + 2] = (real)0;
            }
        }
    }
}

template <typename real>
__device__ __forceinline__ double row_sum(double v)
{
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 16);
    return v;
}

template <typename real, int NS>
__device__ __forceinline__ void load_replica(Regs<real, NS>& r, const real* slab, int n, int l16)
{
    constexpr int npad = 16 * NS;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int a = 16 * s + l16;
        if (a < n) {
            r.x[s] = slab[a];
            r.y[s] = slab[npad + a];
            r.z[s] = slab[2 * npad + a];
            r.vx[s] = slab[3 * npad + a];
            r.vy[s] = slab[4 * npad + a];
            r.vz[s] = slab[5 * npad + a];
        } else {
            // padding atoms: fixed, far apart from the molecule and from each other
            r.x[s] = (real)(1000 + 10 * a);
            r.y[s] = (real)1000;
            r.z[s] = (real)1000;
            r.vx[s] = r.vy[s] = r.vz[s] = (real)0;
        }
    }
}

template <typename real, int NS>
__device__ __forceinline__ void store_replica(const Regs<real, NS>& r, real* slab, int l16)
{
    constexpr int npad = 16 * NS;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int a = 16 * s + l16;
        {
            slab[a] = r.x[s];
            slab[npad + a] = r.y[s];
            slab[2 * npad + a] = r.z[s];
            slab[3 * npad + a] = r.vx[s];
            slab[4 * npad + a] = r.vy[s];
            slab[5 * npad + a] = r.vz[s];
        }
    }
}

// three standard normals from one Philox draw (Box-Muller); the FP32 path
// uses the hardware sine / cosine (argument in revolutions, which is what
// the uniform already is) and logarithm
__device__ __forceinline__ void normals3(const u32x4& w, float* z)
{
    const float s24 = 1.0f / 16777216.0f;
    const float u0 = ((float)(w.v[0] >> 8) + 0.5f) * s24;
    const float u1 = ((float)(w.v[1] >> 8) + 0.5f) * s24;
    const float u2 = ((float)(w.v[2] >> 8) + 0.5f) * s24;
    const float u3 = ((float)(w.v[3] >> 8) + 0.5f) * s24;
    const float ln2 = 0.693147180559945309f;
    const float r0 = __builtin_sqrtf(-2.0f * ln2 * __builtin_amdgcn_logf(u0));
    const float r1 = __builtin_sqrtf(-2.0f * ln2 * __builtin_amdgcn_logf(u2));
    z[0] = r0 * __builtin_amdgcn_cosf(u1);
    z[1] = r0 * __builtin_amdgcn_sinf(u1);
    z[2] = r1 * __builtin_amdgcn_cosf(u3);
}
__device__ __forceinline__ void normals3(const u32x4& w, double* z)
{
    const double s24 = 1.0 / 16777216.0;
    const double u0 = ((double)(w.v[0] >> 8) + 0.5) * s24;
    const double u1 = ((double)(w.v[1] >> 8) + 0.5) * s24;
    const double u2 = ((double)(w.v[2] >> 8) + 0.5) * s24;
    const double u3 = ((double)(w.v[3] >> 8) + 0.5) * s24;
    const double two_pi = 6.283185307179586476925286766559;
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    z[0] = r0 * cos(two_pi * u1);
    z[1] = r0 * sin(two_pi * u1);
    z[2] = r1 * cos(two_pi * u3);
}

// Andersen collisions of one replica at MD step `gstep`: atom a collides iff
// the top 24 bits of its collision word are below p24; its new velocity is
// drawn from Maxwell-Boltzmann at kT (hdtm * two_over_dt = 1 / m)
template <typename real, int NS>
__device__ __forceinline__ void andersen(Regs<real, NS>& r, const RunDev<real>& d, uint32_t slot, uint32_t gstep,
                                         uint32_t p24, real kT, const real* hdtm, real two_over_dt, int l16)
{
#pragma unroll
    for (int q = 0; q < (NS + 3) / 4; ++q) {
        const u32x4 w = philox10(slot, gstep, (uint32_t)(l16 + 16 * q), kStreamCollide, d.key0, d.key1);
#pragma unroll
        for (int s = 4 * q; s < NS && s < 4 * q + 4; ++s) {
            const int a = 16 * s + l16;
            if (a < d.n && (w.v[s & 3] >> 8) < p24) {
                const u32x4 wv = philox10(slot, gstep, (uint32_t)a, kStreamVelocity, d.key0, d.key1);
                real z[3];
                normals3(wv, z);
                const real sd = sqrt_(kT * hdtm[s] * two_over_dt);
                r.vx[s] = sd * z[0];
                r.vy[s] = sd * z[1];
                r.vz[s] = sd * z[2];
            }
        }
    }
}

// Ornstein-Uhlenbeck velocity step of the Langevin bath (the O of B-A-O-A-B):
// v = c1 v + c2 sqrt(kT / m) xi, three normals per atom from stream 5 with
// counter (slot, step, atom, 5)
template <typename real, int NS>
__device__ __forceinline__ void langevin_o(Regs<real, NS>& r, const RunDev<real>& d, uint32_t slot, uint32_t gstep,
                                           real kT, const real* hdtm, real two_over_dt, real c1, real c2, int l16)
{
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int a = 16 * s + l16;
        if (a < d.n) {
            const u32x4 w = philox10(slot, gstep, (uint32_t)a, kStreamLangevin, d.key0, d.key1);
            real z[3];
            normals3(w, z);
            const real sd = c2 * sqrt_(kT * hdtm[s] * two_over_dt);
            r.vx[s] = c1 * r.vx[s] + sd * z[0];
            r.vy[s] = c1 * r.vy[s] + sd * z[1];
            r.vz[s] = c1 * r.vz[s] + sd * z[2];
        }
    }
}

// ---------------------------------------------------------------------------
// the persistent MD kernel (LANG: Langevin bath in the B-A-O-A-B splitting,
// else velocity Verlet with Andersen collisions)
// ---------------------------------------------------------------------------
template <typename real, int NS, int DIEL, int LANG>
__global__ __launch_bounds__(1024) void k_md(RunDev<real> d, int n_steps)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NST = tile_steps(NS);
    real* tab_ab = reinterpret_cast<real*>(smem);
    real* tab_c = tab_ab + NST * 32;
    real* stage = tab_c + NST * 16;
    for (int i = threadIdx.x; i < NST * 32; i += blockDim.x)
        tab_ab[i] = d.nb_ab[i];
    for (int i = threadIdx.x; i < NST * 16; i += blockDim.x)
        tab_c[i] = d.nb_c[i];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int row = lane >> 4;
    const int l16 = lane & 15;
    const int wave = threadIdx.x >> 6;
    real* pos = stage + (size_t)(wave * kRowsPerWave + row) * 6 * d.n;
    real* frc = pos + 3 * d.n;

    const RunCtl* ctl = d.ctl;
    // a run with a sticky error keeps its state (uniform over the launch:
    // only k_md_begin writes `frozen`)
    if (ctl->frozen)
        return;
    const int64_t R = ctl->R_cur;
    const int cur = ctl->cur;
    const uint32_t step0 = ctl->step;
    const real kT = (real)(d.kB * ctl->T_cur);
    const real dt = (real)d.dt;
    real* slab_all = d.slab[cur];
    constexpr int npad = 16 * NS;
    const real two_over_dt = (real)(2.0 / d.dt);

    // per-atom dt / (2 m); 0 for padding atoms, which therefore never move
    real hdtm[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int a = 16 * s + l16;
        hdtm[s] = (a < d.n) ? (real)(0.5 * d.dt / d.mass[a]) : (real)0;
    }
    // the force stage starts cleared
    for (int i = l16; i < 3 * d.n; i += kRow)
        frc[i] = (real)0;

    for (;;) {
        int g = 0;
        if (lane == 0)
            g = atomicAdd(&d.ctl->work, 1);
        g = __builtin_amdgcn_readfirstlane(g);
        const int64_t base = (int64_t)g * kRowsPerWave;
        if (base >= R)
            break;
        const int64_t slot = base + row;
        const bool valid = slot < R;
        const int64_t ls = valid ? slot : base;
        real* slab = slab_all + (size_t)ls * 6 * npad;

        Regs<real, NS> r;
        load_replica<real, NS>(r, slab, d.n, l16);
        double eacc = 0.0;
        // velocity Verlet with the force evaluation at the top of each pass:
        // pass st evaluates F(x_st), finishes step st - 1 (second half kick,
        // collisions) and starts step st (first half kick, drift)
        for (int st = 0; st <= n_steps; ++st) {
            // compiler-only memory barrier: keeps the (step-invariant) term
            // records and pair coefficients from being hoisted out of the step
            // loop into hundreds of live registers
            asm volatile("" ::: "memory");
            evaluate<real, NS, DIEL, false>(r, d, tab_ab, tab_c, pos, frc, l16, eacc);
            if (st > 0) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    r.vx[s] += hdtm[s] * r.fx[s];
                    r.vy[s] += hdtm[s] * r.fy[s];
                    r.vz[s] += hdtm[s] * r.fz[s];
                }
                // Andersen collisions
                if (d.p24 != 0u)
                    andersen<real, NS>(r, d, (uint32_t)ls, step0 + (uint32_t)(st - 1), d.p24, kT, hdtm, two_over_dt,
                                       l16);
            }
            if (st < n_steps) {
                if constexpr (LANG) {
                    const real hdt = (real)(0.5 * d.dt);
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        r.vx[s] += hdtm[s] * r.fx[s];
                        r.vy[s] += hdtm[s] * r.fy[s];
                        r.vz[s] += hdtm[s] * r.fz[s];
                        r.x[s] += hdt * r.vx[s];
                        r.y[s] += hdt * r.vy[s];
                        r.z[s] += hdt * r.vz[s];
                    }
                    langevin_o<real, NS>(r, d, (uint32_t)ls, step0 + (uint32_t)st, kT, hdtm, two_over_dt,
                                         (real)d.lc1, (real)d.lc2, l16);
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        r.x[s] += hdt * r.vx[s];
                        r.y[s] += hdt * r.vy[s];
                        r.z[s] += hdt * r.vz[s];
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        r.vx[s] += hdtm[s] * r.fx[s];
                        r.vy[s] += hdtm[s] * r.fy[s];
                        r.vz[s] += hdtm[s] * r.fz[s];
                        r.x[s] += dt * r.vx[s];
                        r.y[s] += dt * r.vy[s];
                        r.z[s] += dt * r.vz[s];
                    }
                }
            }
        }

        // kinetic energy (FP64) of the final state; the potential energy is
        // evaluated by k_energy after this kernel
        double ek = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int a = 16 * s + l16;
            if (a < d.n) {
                const double vx = r.vx[s], vy = r.vy[s], vz = r.vz[s];
                ek += 0.5 * d.mass[a] * (vx * vx + vy * vy + vz * vz);
            }
        }
        ek = row_sum<real>(ek);
        if (valid) {
            store_replica<real, NS>(r, slab, l16);
            if (l16 == 0)
                d.ekin[cur][slot] = ek;
        }
    }
}

// potential energy (FP64 sum of FP32 terms) of every replica at its current
// positions: E_j of the resampling weights
template <typename real, int NS, int DIEL>
__global__ __launch_bounds__(1024) void k_energy(RunDev<real> d)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NST = tile_steps(NS);
    real* tab_ab = reinterpret_cast<real*>(smem);
    real* tab_c = tab_ab + NST * 32;
    real* stage = tab_c + NST * 16;
    for (int i = threadIdx.x; i < NST * 32; i += blockDim.x)
        tab_ab[i] = d.nb_ab[i];
    for (int i = threadIdx.x; i < NST * 16; i += blockDim.x)
        tab_c[i] = d.nb_c[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, row = lane >> 4, l16 = lane & 15, wave = threadIdx.x >> 6;
    real* pos = stage + (size_t)(wave * kRowsPerWave + row) * 6 * d.n;
    real* frc = pos + 3 * d.n;
    if (d.ctl->frozen)
        return;
    const int64_t R = d.ctl->R_cur;
    const int cur = d.ctl->cur;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; g * kRowsPerWave < R; g += nw) {
        const int64_t slot = g * kRowsPerWave + row;
        const bool valid = slot < R;
        const real* slab = d.slab[cur] + (size_t)(valid ? slot : g * kRowsPerWave) * 6 * (16 * NS);
        Regs<real, NS> r;
        load_replica<real, NS>(r, slab, d.n, l16);
        double ep = 0.0;
        evaluate<real, NS, DIEL, true>(r, d, tab_ab, tab_c, pos, frc, l16, ep);
        ep = row_sum<real>(ep);
        if (valid && l16 == 0) {
            d.epot[cur][slot] = ep;
            if (!isfinite(ep))
                atomicCAS(&d.ctl->error, 0, 4);
        }
    }
}

// forces and energies of replicas [r0, r0 + count) at their current positions
template <typename real, int NS, int DIEL>
__global__ __launch_bounds__(1024) void k_forces(RunDev<real> d, int64_t r0, int count)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NST = tile_steps(NS);
    real* tab_ab = reinterpret_cast<real*>(smem);
    real* tab_c = tab_ab + NST * 32;
    real* stage = tab_c + NST * 16;
    for (int i = threadIdx.x; i < NST * 32; i += blockDim.x)
        tab_ab[i] = d.nb_ab[i];
    for (int i = threadIdx.x; i < NST * 16; i += blockDim.x)
        tab_c[i] = d.nb_c[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, row = lane >> 4, l16 = lane & 15, wave = threadIdx.x >> 6;
    real* pos = stage + (size_t)(wave * kRowsPerWave + row) * 6 * d.n;
    real* frc = pos + 3 * d.n;
    for (int i = l16; i < 3 * d.n; i += kRow)
        frc[i] = (real)0;
    const int cur = d.ctl->cur;
    const int64_t k = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * kRowsPerWave + row;
    const bool valid = k < count;
    const int64_t slot = r0 + (valid ? k : 0);
    const real* slab = d.slab[cur] + (size_t)slot * 6 * (16 * NS);
    Regs<real, NS> r;
    load_replica<real, NS>(r, slab, d.n, l16);
    double dummy = 0.0, ep = 0.0;
    evaluate<real, NS, DIEL, false>(r, d, tab_ab, tab_c, pos, frc, l16, dummy);
    evaluate<real, NS, DIEL, true>(r, d, tab_ab, tab_c, pos, frc, l16, ep);
    ep = row_sum<real>(ep);
    if (valid) {
        double* o = d.dbg + (size_t)k * d.npad * 4;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int a = 16 * s + l16;
            if (a < d.n) {
                o[4 * a] = (double)r.fx[s];
                o[4 * a + 1] = (double)r.fy[s];
                o[4 * a + 2] = (double)r.fz[s];
            }
        }
        if (l16 == 0)
            o[3] = ep;
    }
}

// ---------------------------------------------------------------------------
// r-RESPA pieces for FP32 runs with a learned surrogate (outer step Dt = M dt,
// inner force F_bonded + F_NN, outer impulse F_nb - F_NN).  `ops` selects what
// is applied, in this order, at the current positions:
//   kRespaInnerKick   v += dt/2 (F_b + F_NN) / m      (end of an inner step)
//   kRespaOuterEnd    v += Dt/2 (F_nb - F_NN) / m
//   kRespaCollide     Andersen collisions, step word ctl->step + step_off
//   kRespaOuterStart  v += Dt/2 (F_nb - F_NN) / m
//   kRespaDrift       v += dt/2 (F_b + F_NN) / m; x += dt v  (start of an inner step)
// F_NN comes from `fnn` ([R_cap][3][npad], computed at the current positions);
// F_b and F_nb are evaluated here.  Without kRespaDrift the kinetic energy is stored.
// ---------------------------------------------------------------------------
template <int NS, int DIEL>
__global__ __launch_bounds__(1024) void k_respa(RunDev<float> d, const float* fnn, int ops, uint32_t step_off,
                                                double dt_outer, uint32_t p24_outer)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NST = tile_steps(NS);
    float* tab_ab = reinterpret_cast<float*>(smem);
    float* tab_c = tab_ab + NST * 32;
    float* stage = tab_c + NST * 16;
    for (int i = threadIdx.x; i < NST * 32; i += blockDim.x)
        tab_ab[i] = d.nb_ab[i];
    for (int i = threadIdx.x; i < NST * 16; i += blockDim.x)
        tab_c[i] = d.nb_c[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, row = lane >> 4, l16 = lane & 15, wave = threadIdx.x >> 6;
    float* pos = stage + (size_t)(wave * kRowsPerWave + row) * 6 * d.n;
    float* frc = pos + 3 * d.n;
    for (int i = l16; i < 3 * d.n; i += kRow)
        frc[i] = 0.f;
    const RunCtl* ctl = d.ctl;
    if (ctl->frozen)
        return;
    const int64_t R = ctl->R_cur;
    const int cur = ctl->cur;
    const uint32_t gstep = ctl->step + step_off;
    const float kT = (float)(d.kB * ctl->T_cur);
    const float dt = (float)d.dt;
    const float two_over_dt = (float)(2.0 / d.dt);
    constexpr int npad = 16 * NS;
    float hin[NS], hout[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int a = 16 * s + l16;
        hin[s] = (a < d.n) ? (float)(0.5 * d.dt / d.mass[a]) : 0.f;
        hout[s] = (a < d.n) ? (float)(0.5 * dt_outer / d.mass[a]) : 0.f;
    }
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; g * kRowsPerWave < R; g += nw) {
        const int64_t slot = g * kRowsPerWave + row;
        const bool valid = slot < R;
        const int64_t ls = valid ? slot : g * kRowsPerWave;
        float* slab = d.slab[cur] + (size_t)ls * 6 * npad;
        Regs<float, NS> r;
        load_replica<float, NS>(r, slab, d.n, l16);
        double unused = 0.0;
        evaluate<float, NS, DIEL, false, 1>(r, d, tab_ab, tab_c, pos, frc, l16, unused);
        float bx[NS], by[NS], bz[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            bx[s] = r.fx[s];
            by[s] = r.fy[s];
            bz[s] = r.fz[s];
        }
        if (ops & (kRespaOuterEnd | kRespaOuterStart))
            evaluate<float, NS, DIEL, false, 2>(r, d, tab_ab, tab_c, pos, frc, l16, unused);
        const float* fn = fnn + (size_t)ls * 3 * npad;
        float nx[NS], ny[NS], nz[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int a = 16 * s + l16;
            nx[s] = (a < d.n) ? fn[a] : 0.f;
            ny[s] = (a < d.n) ? fn[npad + a] : 0.f;
            nz[s] = (a < d.n) ? fn[2 * npad + a] : 0.f;
        }
        if (ops & kRespaInnerKick) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                r.vx[s] += hin[s] * (bx[s] + nx[s]);
                r.vy[s] += hin[s] * (by[s] + ny[s]);
                r.vz[s] += hin[s] * (bz[s] + nz[s]);
            }
        }
        if (ops & kRespaOuterEnd) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                r.vx[s] += hout[s] * (r.fx[s] - nx[s]);
                r.vy[s] += hout[s] * (r.fy[s] - ny[s]);
                r.vz[s] += hout[s] * (r.fz[s] - nz[s]);
            }
        }
        if ((ops & kRespaCollide) && p24_outer != 0u)
            andersen<float, NS>(r, d, (uint32_t)ls, gstep, p24_outer, kT, hin, two_over_dt, l16);
        if (ops & kRespaOuterStart) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                r.vx[s] += hout[s] * (r.fx[s] - nx[s]);
                r.vy[s] += hout[s] * (r.fy[s] - ny[s]);
                r.vz[s] += hout[s] * (r.fz[s] - nz[s]);
            }
        }
        if (ops & kRespaDrift) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                r.vx[s] += hin[s] * (bx[s] + nx[s]);
                r.vy[s] += hin[s] * (by[s] + ny[s]);
                r.vz[s] += hin[s] * (bz[s] + nz[s]);
                r.x[s] += dt * r.vx[s];
                r.y[s] += dt * r.vy[s];
                r.z[s] += dt * r.vz[s];
            }
        }
        double ek = 0.0;
        if (!(ops & kRespaDrift)) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int a = 16 * s + l16;
                if (a < d.n) {
                    const double vx = r.vx[s], vy = r.vy[s], vz = r.vz[s];
                    ek += 0.5 * d.mass[a] * (vx * vx + vy * vy + vz * vz);
                }
            }
            ek = row_sum<float>(ek);
        }
        if (valid) {
            store_replica<float, NS>(r, slab, l16);
            if (!(ops & kRespaDrift) && l16 == 0)
                d.ekin[cur][slot] = ek;
        }
    }
}

// positions and exact nonbonded forces of replicas [r0, r0 + count) as
// [count][n][3] FP32 arrays (training data of the surrogate)
template <int NS, int DIEL>
__global__ __launch_bounds__(1024) void k_export(RunDev<float> d, int64_t r0, int64_t count, float* xo, float* fo)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NST = tile_steps(NS);
    float* tab_ab = reinterpret_cast<float*>(smem);
    float* tab_c = tab_ab + NST * 32;
    for (int i = threadIdx.x; i < NST * 32; i += blockDim.x)
        tab_ab[i] = d.nb_ab[i];
    for (int i = threadIdx.x; i < NST * 16; i += blockDim.x)
        tab_c[i] = d.nb_c[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, row = lane >> 4, l16 = lane & 15, wave = threadIdx.x >> 6;
    const int cur = d.ctl->cur;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; g * kRowsPerWave < count; g += nw) {
        const int64_t k = g * kRowsPerWave + row;
        const bool valid = k < count;
        const float* slab = d.slab[cur] + (size_t)(r0 + (valid ? k : g * kRowsPerWave)) * 6 * (16 * NS);
        Regs<float, NS> r;
        load_replica<float, NS>(r, slab, d.n, l16);
        double unused = 0.0;
        evaluate<float, NS, DIEL, false, 2>(r, d, tab_ab, tab_c, nullptr, nullptr, l16, unused);
        if (valid) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int a = 16 * s + l16;
                if (a < d.n) {
                    float* xa = xo + ((size_t)k * d.n + a) * 3;
                    float* fa = fo + ((size_t)k * d.n + a) * 3;
                    xa[0] = r.x[s];
                    xa[1] = r.y[s];
                    xa[2] = r.z[s];
                    fa[0] = r.fx[s];
                    fa[1] = r.fy[s];
                    fa[2] = r.fz[s];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// wide layout: one replica per wavefront (molecules up to 320 atoms, and every
// run of a context that holds one).  Atom a lives on lane a % 64, slot a / 64.
// All-pairs nonbonded forces with Newton's third law: copies of a slot's atoms
// rotate around the wavefront (see wide_evaluate); LJ pair coefficients come
// from the molecule's class table (a copy per wave in LDS), exclusion / 1-4
// bits 64 partners at a time.
// ---------------------------------------------------------------------------
// lane i receives lane (i + 1) mod 64 (DPP wave_rol:1)
__device__ __forceinline__ int wave_rol1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x134, 0xF, 0xF, false); }
__device__ __forceinline__ float wave_rol1(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x134, 0xF, 0xF, false));
}

struct WideRegs {
    float x[kWideSlots], y[kWideSlots], z[kWideSlots];
    float vx[kWideSlots], vy[kWideSlots], vz[kWideSlots];
    float fx[kWideSlots], fy[kWideSlots], fz[kWideSlots];
    float qs[kWideSlots];   // own atoms' Coulomb factors
    int cl[kWideSlots];     // own atoms' LJ classes
};

// a wave's copy of its run's LJ class table (ljsz float2)
__device__ __forceinline__ void wide_load_ljtab(const RunDev<float>& d, float2* lj, int lane, int ljsz)
{
    for (int i = lane; i < ljsz; i += kWide)
        lj[i] = d.ljtab[i];
    wave_sync();
}

// LJ coefficients (12 c12, -6 c6) of a pair from the class table `lj` (this
// wave's LDS copy), its Coulomb factor qs_i qs_j
template <int DIEL, bool ENERGY>
__device__ __forceinline__ void wide_evaluate(WideRegs& r, const RunDev<float>& d, float* pos, float* frc,
                                              const float2* lj, int lane, int nsl, double& eacc)
{
    const int n = d.n;
    if constexpr (!ENERGY) {
#pragma unroll
        for (int s = 0; s < kWideSlots; ++s) {
            r.fx[s] = 0.f;
            r.fy[s] = 0.f;
            r.fz[s] = 0.f;
        }
    }
#pragma unroll
    for (int s = 0; s < kWideSlots; ++s) {
        const int a = kWide * s + lane;
        if (s < nsl && a < n) {
            pos[3 * a] = r.x[s];
            pos[3 * a + 1] = r.y[s];
            pos[3 * a + 2] = r.z[s];
        }
    }
    wave_sync();
    bonded_terms<float, ENERGY, kWide>(d, pos, frc, lane, eacc);
    // Nonbonded pairs, each unordered pair once: for every partner slot t a
    // copy of slot t's atoms (position, Coulomb factor, LJ class column and
    // reaction-force sum) travels around the wavefront one lane per step (DPP
    // wave rotation); at step k lane l holds partner atom 64 t + (l + k) mod 64
    // and pairs it with its own atoms of slots s <= t (same slot: k = 1..32,
    // the k = 32 pair kept on one of its two lanes).  The travelling reaction
    // sums are added to the LDS force stage at the end (distinct atoms per lane).
    const float s14lj = d.s14lj, s14c = d.s14c;
    const char* ljb = reinterpret_cast<const char*>(lj);
    const int row8 = d.lj_stride * (int)sizeof(float2);   // bytes per class-table row
#pragma unroll
    for (int t = 0; t < kWideSlots; ++t) {
        if (t < nsl) {
            float px = r.x[t], py = r.y[t], pz = r.z[t], pqs = r.qs[t];
            int pcl = r.cl[t] * (int)sizeof(float2);   // byte offset of the partner's column
            float pfx = 0.f, pfy = 0.f, pfz = 0.f;
            // own atoms' exclusion / 1-4 bits over the 64 atoms of slot t,
            // rotated so that bit k is the partner met at step k, split into
            // the words of steps k < 32 and k >= 32
            uint32_t exw[kWideSlots][2], s4w[kWideSlots][2];
#pragma unroll
            for (int s = 0; s <= t; ++s) {
                const int a = kWide * s + lane;
                uint64_t ex = ~0ull, s4 = 0ull;
                if (a < n) {
                    uint2 m0 = make_uint2(0u, 0u), m1 = make_uint2(0u, 0u);
                    if (2 * t < d.nchunk)
                        m0 = d.pmask[(size_t)a * d.nchunk + 2 * t];
                    if (2 * t + 1 < d.nchunk)
                        m1 = d.pmask[(size_t)a * d.nchunk + 2 * t + 1];
                    ex = ((uint64_t)m1.x << 32) | m0.x;
                    s4 = ((uint64_t)m1.y << 32) | m0.y;
                }
                ex = (ex >> lane) | (ex << ((kWide - lane) & (kWide - 1)));
                s4 = (s4 >> lane) | (s4 << ((kWide - lane) & (kWide - 1)));
                exw[s][0] = (uint32_t)ex;
                exw[s][1] = (uint32_t)(ex >> 32);
                s4w[s][0] = (uint32_t)s4;
                s4w[s][1] = (uint32_t)(s4 >> 32);
            }
            // steps k at which some lane of own slot s meets an excluded or 1-4
            // partner of slot t (bit k of stepmask[t][s], wave-uniform: held in
            // scalar registers); every other step takes the pair code without
            // masks and scale factors
            uint64_t smask[kWideSlots];
#pragma unroll
            for (int s = 0; s <= t; ++s) {
                const uint64_t m = d.stepmask[t * kWideSlots + s];
                smask[s] = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(m >> 32)) << 32) |
                           (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)m);
            }
            const int kend = (t == 0) ? 33 : kWide;
            // one ring step; h = k / 32 selects the mask words
            auto ring_step = [&](int k, int h) {
                // the pair coefficients of every own slot, read before any of them is used
                float2 ab[kWideSlots];
#pragma unroll
                for (int s = 0; s <= t; ++s)
                    ab[s] = *reinterpret_cast<const float2*>(ljb + (r.cl[s] * row8 + pcl));
                const uint32_t bit = 1u << (k & 31);
#pragma unroll
                for (int s = 0; s <= t; ++s) {
                    if (!(s < t || (k >= 1 && k <= 32)))
                        continue;
                    const float dx = r.x[s] - px, dy = r.y[s] - py, dz = r.z[s] - pz;
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const float ir2 = rcp_(r2);
                    const float ir4 = ir2 * ir2;
                    const float ir6 = ir4 * ir2;
                    const float C = r.qs[s] * pqs;   // Coulomb factor of the pair
                    const float cc = (DIEL == 1) ? ir2 : rsq_(r2);   // Coulomb r-dependence over r^2
                    // g: force on the own atom = g (x_own - x_partner), on the partner
                    // -g (...); u: pair energy.  Only the factors differ between the
                    // plain and the masked step, the updates below are shared.
                    float g = 0.f, u = 0.f;
                    if (!((smask[s] >> k) & 1ull)) {
                        if constexpr (ENERGY)
                            u = ir6 * fma_(ab[s].x * (1.f / 12.f), ir6, ab[s].y * (1.f / 6.f)) +
                                ((DIEL == 1) ? 0.5f * C * ir2 : C * cc);
                        else
                            // g = (12 c12 / r^12 - 6 c6 / r^6 + C c) / r^2, c = 1 / r^2
                            // (dielectric 4r: ((12 c12 / r^6 - 6 c6) / r^4 + C) / r^4)
                            // or 1 / r (vacuum)
                            if constexpr (DIEL == 1)
                                g = fma_(fma_(ab[s].x, ir6, ab[s].y), ir4, C) * ir4;
                            else
                                g = fma_(C, cc, ir6 * fma_(ab[s].x, ir6, ab[s].y)) * ir2;
                    } else {
                        // the same-slot pair at k = 32 is met from both of its lanes:
                        // the upper half of the wave leaves it to the lower
                        const bool skip = (exw[s][h] & bit) != 0u || (s == t && k == 32 && lane >= 32);
                        const bool is14 = (s4w[s][h] & bit) != 0u;
                        const float slj = is14 ? s14lj : 1.f;
                        const float sc = is14 ? s14c : 1.f;
                        if constexpr (ENERGY) {
                            const float ulj = ir6 * fma_(ab[s].x * (1.f / 12.f), ir6, ab[s].y * (1.f / 6.f));
                            const float uc = (DIEL == 1) ? 0.5f * C * ir2 : C * cc;
                            u = skip ? 0.f : slj * ulj + sc * uc;
                        } else {
                            const float t = fma_(ab[s].x, ir6, ab[s].y);
                            const float gg = (DIEL == 1) ? fma_(slj * t, ir4, sc * C) * ir4
                                                         : fma_(sc * C, cc, slj * (ir6 * t)) * ir2;
                            g = skip ? 0.f : gg;
                        }
                    }
                    if constexpr (ENERGY) {
                        eacc += (double)u;
                    } else {
                        r.fx[s] = fma_(g, dx, r.fx[s]);
                        r.fy[s] = fma_(g, dy, r.fy[s]);
                        r.fz[s] = fma_(g, dz, r.fz[s]);
                        pfx = fma_(-g, dx, pfx);
                        pfy = fma_(-g, dy, pfy);
                        pfz = fma_(-g, dz, pfz);
                        // the sums are formed here (an empty asm that reads and writes
                        // them): deferring the updates keeps every slot's displacement
                        // and factor live and spills
                        asm volatile("" : "+v"(r.fx[s]), "+v"(r.fy[s]), "+v"(r.fz[s]), "+v"(pfx), "+v"(pfy),
                                     "+v"(pfz));
                    }
                }
                px = wave_rol1(px);
                py = wave_rol1(py);
                pz = wave_rol1(pz);
                pcl = wave_rol1(pcl);
                pqs = wave_rol1(pqs);
                if constexpr (!ENERGY) {
                    pfx = wave_rol1(pfx);
                    pfy = wave_rol1(pfy);
                    pfz = wave_rol1(pfz);
                }
            };
            for (int k = 0; k < 32; ++k)
                ring_step(k, 0);
            for (int k = 32; k < kend; ++k)
                ring_step(k, 1);
            if constexpr (!ENERGY) {
                // the travelling copy's atom after kend rotations
                const int j = kWide * t + ((lane + kend) & (kWide - 1));
                if (j < n) {
                    frc[3 * j] += pfx;
                    frc[3 * j + 1] += pfy;
                    frc[3 * j + 2] += pfz;
                }
            }
        }
    }
    if constexpr (!ENERGY) {
        wave_sync();
#pragma unroll
        for (int s = 0; s < kWideSlots; ++s) {
            const int a = kWide * s + lane;
            if (s < nsl && a < n) {
                r.fx[s] += frc[3 * a];
                r.fy[s] += frc[3 * a + 1];
                r.fz[s] += frc[3 * a + 2];
                frc[3 * a] = 0.f;
                frc[3 * a + 1] = 0.f;
                frc[3 * a + 2] = 0.f;
            }
        }
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void wide_load(WideRegs& r, const RunDev<float>& d, const float* slab, int lane, int nsl)
{
    const int npad = kWide * nsl;
#pragma unroll
    for (int s = 0; s < kWideSlots; ++s) {
        const int a = kWide * s + lane;
        if (s < nsl && a < d.n) {
            r.x[s] = slab[a];
            r.y[s] = slab[npad + a];
            r.z[s] = slab[2 * npad + a];
            r.vx[s] = slab[3 * npad + a];
            r.vy[s] = slab[4 * npad + a];
            r.vz[s] = slab[5 * npad + a];
            const float2 p = d.apar2[a];
            r.qs[s] = p.x;
            r.cl[s] = (int)p.y;
        } else {
            // padding atoms: fixed, far apart, zero pair parameters (zero LJ class)
            r.x[s] = (float)(1000 + 10 * a);
            r.y[s] = 1000.f;
            r.z[s] = 1000.f;
            r.vx[s] = r.vy[s] = r.vz[s] = 0.f;
            r.qs[s] = 0.f;
            r.cl[s] = d.lj_pad;
        }
    }
}

__device__ __forceinline__ void wide_store(const WideRegs& r, const RunDev<float>& d, float* slab, int lane, int nsl)
{
    const int npad = kWide * nsl;
#pragma unroll
    for (int s = 0; s < kWideSlots; ++s) {
        const int a = kWide * s + lane;
        if (s < nsl && a < d.n) {
            slab[a] = r.x[s];
            slab[npad + a] = r.y[s];
            slab[2 * npad + a] = r.z[s];
            slab[3 * npad + a] = r.vx[s];
            slab[4 * npad + a] = r.vy[s];
            slab[5 * npad + a] = r.vz[s];
        }
    }
}

// Persistent MD of every run of the context in one launch: a device counter
// hands out (run, replica) items, runs in decreasing order of pair work
// (`order`), replicas of a run in slot order.  n_steps velocity-Verlet steps
// with Andersen collisions, then E_pot (FP64 sum) and E_kin of the final state.
// LDS: per wave the position and force stage [2][nmax][3]; after those, per
// wave its copy of its current run's LJ class table (ljsz float2, the
// context's table shape).  128 VGPRs: four waves per SIMD when the LDS allows.
template <int DIEL, int LANG>
__global__ __launch_bounds__(256, 4) void k_md_wide(const RunDev<float>* runs, const int32_t* order, int n_runs,
                                                  int32_t* counter, int nmax, int n_steps, int ljsz)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float* pos = reinterpret_cast<float*>(smem) + (size_t)wave * 6 * nmax;
    float* frc = pos + 3 * nmax;
    float2* lj = reinterpret_cast<float2*>(reinterpret_cast<float*>(smem) + (size_t)(blockDim.x >> 6) * 6 * nmax) +
                 wave * ljsz;
    for (int i = lane; i < 3 * nmax; i += kWide)
        frc[i] = 0.f;
    int lj_run = -1;   // run whose class table the wave holds
    for (;;) {
        int g = 0;
        if (lane == 0)
            g = atomicAdd(counter, 1);
        g = __builtin_amdgcn_readfirstlane(g);
        int k = -1;
        int64_t rep = g;
        for (int q = 0; q < n_runs; ++q) {
            const int run = order[q];
            // frozen runs (sticky error at the start of the call) hand out no items
            const int64_t R = runs[run].ctl->frozen ? 0 : runs[run].ctl->R_cur;
            if (rep < R) {
                k = run;
                break;
            }
            rep -= R;
        }
        k = __builtin_amdgcn_readfirstlane(k);
        if (k < 0)
            break;
        const RunDev<float>& d = runs[k];
        if (k != lj_run) {
            wide_load_ljtab(d, lj, lane, ljsz);
            lj_run = k;
        }
        const int nsl = (d.n + kWide - 1) / kWide;
        const int npad = kWide * nsl;
        const RunCtl* ctl = d.ctl;
        const int cur = ctl->cur;
        const uint32_t step0 = ctl->step;
        const float kT = (float)(d.kB * ctl->T_cur);
        const float dt = (float)d.dt;
        const float two_over_dt = (float)(2.0 / d.dt);
        float* slab = d.slab[cur] + (size_t)rep * 6 * npad;
        float hdtm[kWideSlots];
#pragma unroll
        for (int s = 0; s < kWideSlots; ++s) {
            const int a = kWide * s + lane;
            hdtm[s] = (s < nsl && a < d.n) ? (float)(0.5 * d.dt / d.mass[a]) : 0.f;
        }
        WideRegs r;
        wide_load(r, d, slab, lane, nsl);
        double unused = 0.0;
        for (int st = 0; st <= n_steps; ++st) {
            wide_evaluate<DIEL, false>(r, d, pos, frc, lj, lane, nsl, unused);
            if (st > 0) {
#pragma unroll
                for (int s = 0; s < kWideSlots; ++s) {
                    r.vx[s] += hdtm[s] * r.fx[s];
                    r.vy[s] += hdtm[s] * r.fy[s];
                    r.vz[s] += hdtm[s] * r.fz[s];
                }
                if (d.p24 != 0u) {
                    const uint32_t gstep = step0 + (uint32_t)(st - 1);
#pragma unroll
                    for (int s = 0; s < kWideSlots; ++s) {
                        const int a = kWide * s + lane;
                        if (s < nsl && a < d.n) {
                            const u32x4 w = philox10((uint32_t)rep, gstep, (uint32_t)((a & 15) + 16 * (a >> 6)),
                                                     kStreamCollide, d.key0, d.key1);
                            const int q = (a >> 4) & 3;
                            const uint32_t wq = q == 0 ? w.v[0] : q == 1 ? w.v[1] : q == 2 ? w.v[2] : w.v[3];
                            if ((wq >> 8) < d.p24) {
                                const u32x4 wv = philox10((uint32_t)rep, gstep, (uint32_t)a, kStreamVelocity, d.key0,
                                                          d.key1);
                                float zz[3];
                                normals3(wv, zz);
                                const float sd = sqrt_(kT * hdtm[s] * two_over_dt);
                                r.vx[s] = sd * zz[0];
                                r.vy[s] = sd * zz[1];
                                r.vz[s] = sd * zz[2];
                            }
                        }
                    }
                }
            }
            if (st < n_steps) {
                if constexpr (LANG) {
                    // B-A-O-A-B: half kick, half drift, OU step, half drift
                    const float hdt = (float)(0.5 * d.dt);
                    const float c1 = (float)d.lc1, c2 = (float)d.lc2;
                    const uint32_t gstep = step0 + (uint32_t)st;
#pragma unroll
                    for (int s = 0; s < kWideSlots; ++s) {
                        r.vx[s] += hdtm[s] * r.fx[s];
                        r.vy[s] += hdtm[s] * r.fy[s];
                        r.vz[s] += hdtm[s] * r.fz[s];
                        r.x[s] += hdt * r.vx[s];
                        r.y[s] += hdt * r.vy[s];
                        r.z[s] += hdt * r.vz[s];
                        const int a = kWide * s + lane;
                        if (s < nsl && a < d.n) {
                            const u32x4 w = philox10((uint32_t)rep, gstep, (uint32_t)a, kStreamLangevin, d.key0,
                                                     d.key1);
                            float zz[3];
                            normals3(w, zz);
                            const float sd = c2 * sqrt_(kT * hdtm[s] * two_over_dt);
                            r.vx[s] = c1 * r.vx[s] + sd * zz[0];
                            r.vy[s] = c1 * r.vy[s] + sd * zz[1];
                            r.vz[s] = c1 * r.vz[s] + sd * zz[2];
                        }
                        r.x[s] += hdt * r.vx[s];
                        r.y[s] += hdt * r.vy[s];
                        r.z[s] += hdt * r.vz[s];
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < kWideSlots; ++s) {
                        r.vx[s] += hdtm[s] * r.fx[s];
                        r.vy[s] += hdtm[s] * r.fy[s];
                        r.vz[s] += hdtm[s] * r.fz[s];
                        r.x[s] += dt * r.vx[s];
                        r.y[s] += dt * r.vy[s];
                        r.z[s] += dt * r.vz[s];
                    }
                }
            }
        }
        double ep = 0.0, ek = 0.0;
        wide_evaluate<DIEL, true>(r, d, pos, frc, lj, lane, nsl, ep);
#pragma unroll
        for (int s = 0; s < kWideSlots; ++s) {
            const int a = kWide * s + lane;
            if (s < nsl && a < d.n) {
                const double vx = r.vx[s], vy = r.vy[s], vz = r.vz[s];
                ek += 0.5 * d.mass[a] * (vx * vx + vy * vy + vz * vz);
            }
        }
        ep = wave_sum(ep);
        ek = wave_sum(ek);
        wide_store(r, d, slab, lane, nsl);
        if (lane == 0) {
            d.epot[cur][rep] = ep;
            d.ekin[cur][rep] = ek;
            if (!isfinite(ep))
                atomicCAS(&d.ctl->error, 0, 4);
        }
    }
}

// start of a batched MD call: every run of the launch (order[0 .. n_runs))
// whose sticky error is set stays frozen for the whole call
__global__ void k_wide_begin(RunDev<float>* runs, const int32_t* order, int n_runs)
{
    for (int q = threadIdx.x; q < n_runs; q += blockDim.x)
        runs[order[q]].ctl->frozen = runs[order[q]].ctl->error != 0;
}

// reset of the batch work counter and the step counter of every run of the
// launch after k_md_wide
__global__ void k_wide_finalize(RunDev<float>* runs, const int32_t* order, int n_runs, int32_t* counter,
                                int n_steps)
{
    if (threadIdx.x != 0)
        return;
    *counter = 0;
    for (int q = 0; q < n_runs; ++q) {
        RunCtl* ctl = runs[order[q]].ctl;
        if (!ctl->frozen)
            ctl->step += (uint32_t)n_steps;
        ctl->work = 0;
    }
}

// forces and energies of replicas [r0, r0 + count) of one wide-layout run
template <int DIEL>
__global__ __launch_bounds__(512) void k_forces_wide(RunDev<float> d, int64_t r0, int count, int nmax, int ljsz)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float* pos = reinterpret_cast<float*>(smem) + (size_t)wave * 6 * nmax;
    float* frc = pos + 3 * nmax;
    float2* lj = reinterpret_cast<float2*>(reinterpret_cast<float*>(smem) + (size_t)(blockDim.x >> 6) * 6 * nmax) +
                 wave * ljsz;
    for (int i = lane; i < 3 * nmax; i += kWide)
        frc[i] = 0.f;
    const int k = blockIdx.x * (blockDim.x >> 6) + wave;
    if (k >= count)
        return;
    wide_load_ljtab(d, lj, lane, ljsz);
    const int nsl = (d.n + kWide - 1) / kWide;
    const float* slab = d.slab[d.ctl->cur] + (size_t)(r0 + k) * 6 * kWide * nsl;
    WideRegs r;
    wide_load(r, d, slab, lane, nsl);
    double unused = 0.0, ep = 0.0;
    wide_evaluate<DIEL, false>(r, d, pos, frc, lj, lane, nsl, unused);
    wide_evaluate<DIEL, true>(r, d, pos, frc, lj, lane, nsl, ep);
    ep = wave_sum(ep);
    double* o = d.dbg + (size_t)k * d.npad * 4;
#pragma unroll
    for (int s = 0; s < kWideSlots; ++s) {
        const int a = kWide * s + lane;
        if (s < nsl && a < d.n) {
            o[4 * a] = (double)r.fx[s];
            o[4 * a + 1] = (double)r.fy[s];
            o[4 * a + 2] = (double)r.fz[s];
        }
    }
    if (lane == 0)
        o[3] = ep;
}

// ---------------------------------------------------------------------------
// host-side dispatch
// ---------------------------------------------------------------------------
template <typename real>
size_t md_lds_bytes(int nslot, int n, int waves)
{
    return (size_t)tile_steps(nslot) * 16 * 3 * sizeof(real) + (size_t)waves * kRowsPerWave * 6 * n * sizeof(real);
}

template <typename real, int NS, int DIEL>
static hipError_t launch_md_t(const RunDev<real>& d, int n_steps, int blocks, int waves, hipStream_t s)
{
    const size_t lds = md_lds_bytes<real>(NS, d.n, waves);
    if (d.thermostat == PAMD_THERMOSTAT_LANGEVIN)
        hipLaunchKernelGGL((k_md<real, NS, DIEL, 1>), dim3(blocks), dim3(waves * 64), lds, s, d, n_steps);
    else
        hipLaunchKernelGGL((k_md<real, NS, DIEL, 0>), dim3(blocks), dim3(waves * 64), lds, s, d, n_steps);
    return hipGetLastError();
}

template <typename real, int NS, int DIEL>
static hipError_t launch_energy_t(const RunDev<real>& d, int blocks, int waves, hipStream_t s)
{
    const size_t lds = md_lds_bytes<real>(NS, d.n, waves);
    hipLaunchKernelGGL((k_energy<real, NS, DIEL>), dim3(blocks), dim3(waves * 64), lds, s, d);
    return hipGetLastError();
}

template <typename real, int NS, int DIEL>
static hipError_t launch_forces_t(const RunDev<real>& d, int64_t r0, int count, int waves, hipStream_t s)
{
    const size_t lds = md_lds_bytes<real>(NS, d.n, waves);
    const int per_block = waves * kRowsPerWave;
    const int blocks = (count + per_block - 1) / per_block;
    hipLaunchKernelGGL((k_forces<real, NS, DIEL>), dim3(blocks), dim3(waves * 64), lds, s, d, r0, count);
    return hipGetLastError();
}

template <int NS, int DIEL>
static hipError_t launch_respa_t(const RunDev<float>& d, const float* fnn, int ops, uint32_t step_off,
                                 double dt_outer, uint32_t p24_outer, int blocks, int waves, hipStream_t s)
{
    const size_t lds = md_lds_bytes<float>(NS, d.n, waves);
    hipLaunchKernelGGL((k_respa<NS, DIEL>), dim3(blocks), dim3(waves * 64), lds, s, d, fnn, ops, step_off, dt_outer,
                       p24_outer);
    return hipGetLastError();
}

template <int NS, int DIEL>
static hipError_t launch_export_t(const RunDev<float>& d, int64_t r0, int64_t count, float* xo, float* fo,
                                  int waves, hipStream_t s)
{
    const size_t lds = md_lds_bytes<float>(NS, d.n, waves);
    const int64_t per_block = (int64_t)waves * kRowsPerWave;
    const int64_t blocks = (count + per_block - 1) / per_block;
    hipLaunchKernelGGL((k_export<NS, DIEL>), dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(waves * 64),
                       lds, s, d, r0, count, xo, fo);
    return hipGetLastError();
}

// one-time set-up of an instantiation: LDS limit of its three kernels (outside
// any stream capture) and the resident workgroups per CU of k_md
template <typename real, int NS, int DIEL>
static hipError_t occupancy_t(int waves, int* blocks_per_cu, int n)
{
    const size_t lds = md_lds_bytes<real>(NS, n, waves);
    const void* fns[6] = {(const void*)k_md<real, NS, DIEL, 0>, (const void*)k_energy<real, NS, DIEL>,
                          (const void*)k_forces<real, NS, DIEL>, (const void*)k_md<real, NS, DIEL, 1>, nullptr,
                          nullptr};
    if constexpr (sizeof(real) == 4) {
        fns[4] = (const void*)k_respa<NS, DIEL>;
        fns[5] = (const void*)k_export<NS, DIEL>;
    }
    for (const void* f : fns) {
        if (!f)
            continue;
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    // the Langevin variant needs a few more registers: the smaller occupancy of the two
    int b0 = 0, b1 = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b0, (const void*)k_md<real, NS, DIEL, 0>,
                                                                waves * 64, lds);
    if (e != hipSuccess)
        return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, (const void*)k_md<real, NS, DIEL, 1>, waves * 64, lds);
    *blocks_per_cu = b0 < b1 ? b0 : b1;
    return e;
}

#define PAMD_DISPATCH(REAL, NSV, DIELV, CALL)                                                    \
    switch (NSV * 2 + DIELV) {                                                                  \
    case 1 * 2 + 0: return CALL(REAL, 1, 0);                                                    \
    case 1 * 2 + 1: return CALL(REAL, 1, 1);                                                    \
    case 2 * 2 + 0: return CALL(REAL, 2, 0);                                                    \
    case 2 * 2 + 1: return CALL(REAL, 2, 1);                                                    \
    case 3 * 2 + 0: return CALL(REAL, 3, 0);                                                    \
    case 3 * 2 + 1: return CALL(REAL, 3, 1);                                                    \
    case 4 * 2 + 0: return CALL(REAL, 4, 0);                                                    \
    case 4 * 2 + 1: return CALL(REAL, 4, 1);                                                    \
    case 5 * 2 + 0: return CALL(REAL, 5, 0);                                                    \
    case 5 * 2 + 1: return CALL(REAL, 5, 1);                                                    \
    default: return hipErrorInvalidValue;                                                       \
    }

#define PAMD_DISPATCH64(NSV, DIELV, CALL)                                                        \
    switch (NSV * 2 + DIELV) {                                                                  \
    case 1 * 2 + 0: return CALL(double, 1, 0);                                                  \
    case 1 * 2 + 1: return CALL(double, 1, 1);                                                  \
    case 2 * 2 + 0: return CALL(double, 2, 0);                                                  \
    case 2 * 2 + 1: return CALL(double, 2, 1);                                                  \
    default: return hipErrorInvalidValue;                                                       \
    }

hipError_t launch_md(const RunDev<float>& d, int n_steps, int blocks, int waves, hipStream_t s)
{
#define CALL(R, N, D) launch_md_t<R, N, D>(d, n_steps, blocks, waves, s)
    PAMD_DISPATCH(float, d.nslot, d.dielectric, CALL)
#undef CALL
}
hipError_t launch_md(const RunDev<double>& d, int n_steps, int blocks, int waves, hipStream_t s)
{
#define CALL(R, N, D) launch_md_t<R, N, D>(d, n_steps, blocks, waves, s)
    PAMD_DISPATCH64(d.nslot, d.dielectric, CALL)
#undef CALL
}
hipError_t launch_energy(const RunDev<float>& d, int blocks, int waves, hipStream_t s)
{
#define CALL(R, N, D) launch_energy_t<R, N, D>(d, blocks, waves, s)
    PAMD_DISPATCH(float, d.nslot, d.dielectric, CALL)
#undef CALL
}
hipError_t launch_energy(const RunDev<double>& d, int blocks, int waves, hipStream_t s)
{
#define CALL(R, N, D) launch_energy_t<R, N, D>(d, blocks, waves, s)
    PAMD_DISPATCH64(d.nslot, d.dielectric, CALL)
#undef CALL
}
hipError_t launch_forces(const RunDev<float>& d, int64_t r0, int count, int waves, hipStream_t s)
{
#define CALL(R, N, D) launch_forces_t<R, N, D>(d, r0, count, waves, s)
    PAMD_DISPATCH(float, d.nslot, d.dielectric, CALL)
#undef CALL
}
hipError_t launch_forces(const RunDev<double>& d, int64_t r0, int count, int waves, hipStream_t s)
{
#define CALL(R, N, D) launch_forces_t<R, N, D>(d, r0, count, waves, s)
    PAMD_DISPATCH64(d.nslot, d.dielectric, CALL)
#undef CALL
}
hipError_t launch_respa(const RunDev<float>& d, const float* fnn, int ops, uint32_t step_off, double dt_outer,
                        uint32_t p24_outer, int blocks, int waves, hipStream_t s)
{
#define CALL(R, N, D) launch_respa_t<N, D>(d, fnn, ops, step_off, dt_outer, p24_outer, blocks, waves, s)
    PAMD_DISPATCH(float, d.nslot, d.dielectric, CALL)
#undef CALL
}
hipError_t launch_export(const RunDev<float>& d, int64_t r0, int64_t count, float* xo, float* fo, int waves,
                         hipStream_t s)
{
#define CALL(R, N, D) launch_export_t<N, D>(d, r0, count, xo, fo, waves, s)
    PAMD_DISPATCH(float, d.nslot, d.dielectric, CALL)
#undef CALL
}
size_t wide_lds_bytes(int nmax, int waves, int ljsz)
{
    return (size_t)waves * (6 * nmax * sizeof(float) + ljsz * sizeof(float2));
}

hipError_t wide_setup(int diel, int nmax, int waves, int ljsz, int* blocks_per_cu)
{
    const size_t lds = wide_lds_bytes(nmax, waves, ljsz);
    const void* md = diel ? (const void*)k_md_wide<1, 0> : (const void*)k_md_wide<0, 0>;
    const void* ml = diel ? (const void*)k_md_wide<1, 1> : (const void*)k_md_wide<0, 1>;
    const void* fo = diel ? (const void*)k_forces_wide<1> : (const void*)k_forces_wide<0>;
    for (const void* f : {md, ml, fo}) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    int b0 = 0, b1 = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b0, md, waves * 64, lds);
    if (e != hipSuccess)
        return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, ml, waves * 64, lds);
    *blocks_per_cu = b0 < b1 ? b0 : b1;
    return e;
}

hipError_t launch_md_wide(const RunDev<float>* runs, const int32_t* order, int n_runs, int32_t* counter, int nmax,
                          int n_steps, int diel, int lang, int ljsz, int blocks, int waves, hipStream_t s)
{
    const size_t lds = wide_lds_bytes(nmax, waves, ljsz);
    const dim3 g(blocks), b(waves * 64);
    hipLaunchKernelGGL(k_wide_begin, dim3(1), dim3(64), 0, s, const_cast<RunDev<float>*>(runs), order, n_runs);
    switch (diel * 2 + lang) {
    case 0: hipLaunchKernelGGL((k_md_wide<0, 0>), g, b, lds, s, runs, order, n_runs, counter, nmax, n_steps, ljsz); break;
    case 1: hipLaunchKernelGGL((k_md_wide<0, 1>), g, b, lds, s, runs, order, n_runs, counter, nmax, n_steps, ljsz); break;
    case 2: hipLaunchKernelGGL((k_md_wide<1, 0>), g, b, lds, s, runs, order, n_runs, counter, nmax, n_steps, ljsz); break;
    default: hipLaunchKernelGGL((k_md_wide<1, 1>), g, b, lds, s, runs, order, n_runs, counter, nmax, n_steps, ljsz); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_wide_finalize, dim3(1), dim3(64), 0, s, const_cast<RunDev<float>*>(runs), order, n_runs,
                       counter, n_steps);
    return hipGetLastError();
}

hipError_t launch_forces_wide(const RunDev<float>& d, int64_t r0, int count, int nmax, int waves, int ljsz,
                              hipStream_t s)
{
    const size_t lds = wide_lds_bytes(nmax, waves, ljsz);
    const int blocks = (count + waves - 1) / waves;
    if (d.dielectric)
        hipLaunchKernelGGL(k_forces_wide<1>, dim3(blocks), dim3(waves * 64), lds, s, d, r0, count, nmax, ljsz);
    else
        hipLaunchKernelGGL(k_forces_wide<0>, dim3(blocks), dim3(waves * 64), lds, s, d, r0, count, nmax, ljsz);
    return hipGetLastError();
}

hipError_t md_occupancy(int precision_fp32, int nslot, int diel, int n, int waves, int* blocks_per_cu)
{
    if (precision_fp32) {
#define CALL(R, N, D) occupancy_t<R, N, D>(waves, blocks_per_cu, n)
        PAMD_DISPATCH(float, nslot, diel, CALL)
#undef CALL
    } else {
#define CALL(R, N, D) occupancy_t<R, N, D>(waves, blocks_per_cu, n)
        PAMD_DISPATCH64(nslot, diel, CALL)
#undef CALL
    }
}
size_t md_lds(int precision_fp32, int nslot, int n, int waves)
{
    return precision_fp32 ? md_lds_bytes<float>(nslot, n, waves) : md_lds_bytes<double>(nslot, n, waves);
}

}  // namespace pamd
