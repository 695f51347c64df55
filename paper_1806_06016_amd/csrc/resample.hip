// PAMD steps 1, 2 and 4 on gfx950: initial population, Boltzmann resampling
// and population observables.
//
//   weights   tau_j = exp(-(1/kB T_i - 1/kB T_{i-1}) E_j) / Q,
//             Q = (1/R) sum_j exp(-(1/kB T_i - 1/kB T_{i-1}) E_j)        (PAMD scheme, step 2)
//             evaluated as m = min E, S = sum exp(-dbeta (E - m)), ln Q = -dbeta m + ln S - ln R;
//             ln Q_i estimates ln Z(T_i) - ln Z(T_{i-1}) and is summed on the device
//   adaptive  T_i: the step whose normalised weight variance R sum p^2 - 1
//             equals the target, by safeguarded Newton iterations on dbeta
//   counts    nearest: c_j = floor(tau_j) + [u_j < frac(tau_j)], tau_j = R_target w_j / S;
//             multinomial: R_target independent draws from p_j = w_j / S (the rule
//             stated after the scheme), each an inverse-CDF binary search over
//             the FP64 running sums W_j; none: c_j = 1
//   scan      exclusive prefix sum of c -> destination slots, copies of source
//             j in consecutive slots in increasing j
//   gather    slab copy into the other ping-pong buffer, velocities scaled by
//             sqrt(T_i / T_{i-1}), centre of mass translated to the origin
//
// All reductions run in FP64 in a fixed order (one 1024-thread workgroup per
// run, strided per-thread sums then a tree), so results do not depend on
// scheduling.  The gather is HBM bound: one wavefront per destination slab.
#include <math.h>

#include "pamd.h"
#include "pamd_internal.h"
#include "philox.h"

namespace pamd {

constexpr int kBlk = 1024;

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int o = kBlk / 2; o > 0; o >>= 1) {
        if (t < o)
            sh[t] += sh[t + o];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_min(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int o = kBlk / 2; o > 0; o >>= 1) {
        if (t < o)
            sh[t] = fmin(sh[t], sh[t + o]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// exclusive scan of one int64 per thread; returns the thread's offset, *total the sum
__device__ __forceinline__ int64_t block_exscan(int64_t v, int64_t* sh, int64_t* total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    // Hillis-Steele inclusive scan
    for (int o = 1; o < kBlk; o <<= 1) {
        const int64_t add = (t >= o) ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const int64_t inc = sh[t];
    *total = sh[kBlk - 1];
    __syncthreads();
    return inc - v;
}

// S = sum w, S1 = sum w e, S2 = sum w^2, S21 = sum w^2 e with e = E - m and
// w = exp(-db e), fixed order
__device__ __forceinline__ void weight_moments(const double* E, int64_t R, double db, double m, double* sh,
                                               double* S, double* S1, double* S2, double* S21)
{
    double s = 0.0, s1 = 0.0, s2 = 0.0, s21 = 0.0;
    for (int64_t j = threadIdx.x; j < R; j += kBlk) {
        const double e = E[j] - m;
        const double w = exp(-db * e);
        const double ww = w * w;
        s += w;
        s1 += w * e;
        s2 += ww;
        s21 += ww * e;
    }
    *S = block_sum(s, sh);
    *S1 = block_sum(s1, sh);
    *S2 = block_sum(s2, sh);
    *S21 = block_sum(s21, sh);
}

// sums S = sum w, S2 = sum w^2 with w = exp(-db (E - m)), fixed order
__device__ __forceinline__ void weight_sums(const double* E, int64_t R, double db, double m, double* sh,
                                            double* S, double* S2)
{
    double s = 0.0, s2 = 0.0;
    for (int64_t j = threadIdx.x; j < R; j += kBlk) {
        const double w = exp(-db * (E[j] - m));
        s += w;
        s2 += w * w;
    }
    *S = block_sum(s, sh);
    *S2 = block_sum(s2, sh);
}

// --------------------------------------------------------------------------
// PAMD step 1: initial population
// --------------------------------------------------------------------------
template <typename real>
__global__ void k_init(RunDev<real> d)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = d.R_target * (int64_t)d.npad;
    if (gid == 0) {
        RunCtl* c = d.ctl;
        c->T_cur = d.T0;
        c->T_prev = d.T0;
        c->T_next = d.T0;
        c->T_req = 0.0;
        c->dbeta = c->m = c->S = c->S2 = 0.0;
        c->lnQ_last = c->sum_lnQ = 0.0;
        c->V_last = 0.0;
        c->R_cur = d.R_target;
        c->R_new = d.R_target;
        c->R_prev = d.R_target;
        c->step = 0;
        c->temp_index = 0;
        c->cur = 0;
        c->error = 0;
        c->work = 0;
        c->frozen = 0;
    }
    if (gid >= total)
        return;
    const int64_t r = gid / d.npad;
    const int a = (int)(gid % d.npad);
    real* slab = d.slab[0] + (size_t)r * 6 * d.npad;
    if (a < d.n) {
        const u32x4 w = philox10((uint32_t)r, 0u, (uint32_t)a, kStreamInit, d.key0, d.key1);
        const double s24 = 1.0 / 16777216.0;
        const double u0 = ((double)(w.v[0] >> 8) + 0.5) * s24, u1 = ((double)(w.v[1] >> 8) + 0.5) * s24;
        const double u2 = ((double)(w.v[2] >> 8) + 0.5) * s24, u3 = ((double)(w.v[3] >> 8) + 0.5) * s24;
        const double two_pi = 6.283185307179586476925286766559;
        const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
        const double sd = sqrt(d.kB * d.T0 / d.mass[a]);
        slab[a] = (real)d.x_init[3 * a];
        slab[d.npad + a] = (real)d.x_init[3 * a + 1];
        slab[2 * d.npad + a] = (real)d.x_init[3 * a + 2];
        slab[3 * d.npad + a] = (real)(sd * r0 * cos(two_pi * u1));
        slab[4 * d.npad + a] = (real)(sd * r0 * sin(two_pi * u1));
        slab[5 * d.npad + a] = (real)(sd * r1 * cos(two_pi * u3));
    } else {
        slab[a] = (real)(1000 + 10 * a);
        slab[d.npad + a] = (real)1000;
        slab[2 * d.npad + a] = (real)1000;
        slab[3 * d.npad + a] = slab[4 * d.npad + a] = slab[5 * d.npad + a] = (real)0;
    }
    if (a == 0) {
        d.anc[0][r] = (int32_t)r;
        d.epot[0][r] = 0.0;
        d.ekin[0][r] = 0.0;
    }
}

// --------------------------------------------------------------------------
// PAMD step 2a: minimum, adaptive temperature, normaliser
// --------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(kBlk) void k_weights(RunDev<real> d, double T_req)
{
    __shared__ double sh[kBlk];
    RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t R = c->R_cur;
    const double* E = d.epot[c->cur];
    const double kB = d.kB;
    const double T = c->T_cur;
    double mn = INFINITY, bad = 0.0;
    for (int64_t j = threadIdx.x; j < R; j += kBlk) {
        const double e = E[j];
        if (!isfinite(e))
            bad = 1.0;
        mn = fmin(mn, e);
    }
    mn = block_min(mn, sh);
    bad = block_sum(bad, sh);
    if (bad > 0.0) {
        if (threadIdx.x == 0)
            atomicCAS(&c->error, 0, 4);
        return;
    }
    double Tn;
    if (T_req > 0.0) {
        Tn = T_req;
    } else if (T_req < 0.0) {
        // device schedule: the next entry, or stay at the last one
        const int64_t nx = (int64_t)c->temp_index + 1;
        Tn = (d.sched && nx < d.n_sched) ? d.sched[nx] : T;
    } else {
        const double dmax = 1.0 / (kB * d.T_final) - 1.0 / (kB * T);
        if (!(dmax > 0.0)) {
            Tn = T;
        } else {
            double S, S2;
            weight_sums(E, R, dmax, mn, sh, &S, &S2);
            if ((double)R * S2 / (S * S) - 1.0 <= d.V_target) {
                Tn = d.T_final;
            } else {
                // root of V(b) = V_target in (0, dmax) (V grows with b): Newton
                // steps on V, each one O(R) pass for S, S1 = sum w e, S2 and
                // S21 = sum w^2 e (e = E - m), dV/db = 2 R (S2 S1 / S^3 - S21 / S^2);
                // a step leaving the bracket [lo, hi] bisects instead.  Start:
                // the Gaussian-energy solution sqrt(ln(1 + V_target)) / std(E).
                double lo = 0.0, hi = dmax;
                double e1 = 0.0, e2 = 0.0;
                for (int64_t j = threadIdx.x; j < R; j += kBlk) {
                    const double e = E[j] - mn;
                    e1 += e;
                    e2 += e * e;
                }
                e1 = block_sum(e1, sh) / (double)R;
                e2 = block_sum(e2, sh) / (double)R;
                const double var = e2 - e1 * e1;
                double b = var > 0.0 ? sqrt(log1p(d.V_target) / var) : 0.5 * dmax;
                if (!(b > lo && b < hi))
                    b = 0.5 * (lo + hi);
                for (int it = 0; it < 64; ++it) {
                    double S1, S21;
                    weight_moments(E, R, b, mn, sh, &S, &S1, &S2, &S21);
                    const double V = (double)R * S2 / (S * S) - 1.0;
                    if (V <= d.V_target)
                        lo = b;
                    else
                        hi = b;
                    const double dV = 2.0 * (double)R * (S2 * S1 / (S * S * S) - S21 / (S * S));
                    double bn = b - (V - d.V_target) / dV;
                    if (!(bn > lo && bn < hi))
                        bn = 0.5 * (lo + hi);
                    const bool done = fabs(bn - b) <= 1e-13 * b || hi - lo <= 1e-12 * hi;
                    b = bn;
                    if (done)
                        break;
                }
                Tn = 1.0 / (kB * (b + 1.0 / (kB * T)));
            }
        }
    }
    const double db = 1.0 / (kB * Tn) - 1.0 / (kB * T);
    double S, S2;
    weight_sums(E, R, db, mn, sh, &S, &S2);
    if (threadIdx.x == 0) {
        c->T_req = T_req;
        c->T_next = Tn;
        c->dbeta = db;
        c->m = mn;
        c->S = S;
        c->S2 = S2;
        c->lnQ_last = -db * mn + log(S) - log((double)R);
        c->V_last = (double)R * S2 / (S * S) - 1.0;
    }
}

// --------------------------------------------------------------------------
// Multinomial resampling, part 1: running weight sums W_j = w_0 + ... + w_j
// in FP64 and zeroed counts.  Thread t sums its chunk left to right; the
// chunk totals are scanned serially, and W_j = offset_t + (partial sum of the
// chunk up to j), so W is non-decreasing (rounding is monotone and the last
// W of a chunk equals the next chunk's offset) and zero weights leave it flat.
// --------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(kBlk) void k_cdf(RunDev<real> d)
{
    __shared__ double sh[kBlk];
    const RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t R = c->R_cur;
    const double* E = d.epot[c->cur];
    const double db = c->dbeta, m = c->m;
    const int64_t chunk = (R + kBlk - 1) / kBlk;
    const int64_t j0 = (int64_t)threadIdx.x * chunk;
    const int64_t j1 = (j0 + chunk < R) ? j0 + chunk : R;
    double part = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        part += exp(-db * (E[j] - m));
        d.cdf[j] = part;
        d.counts[j] = 0;
    }
    sh[threadIdx.x] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int t = 0; t < kBlk; ++t) {
            const double p = sh[t];
            sh[t] = run;
            run += p;
        }
    }
    __syncthreads();
    const double off = sh[threadIdx.x];
    for (int64_t j = j0; j < j1; ++j)
        d.cdf[j] = off + d.cdf[j];
}

// Multinomial resampling, part 2: one thread per draw k < R_target picks the
// first j with W_j > u_k W_{R-1} (if rounding leaves none, the first j with
// W_j >= u_k W_{R-1}) by binary search and adds one copy of j.
template <typename real>
__global__ __launch_bounds__(256) void k_draw(RunDev<real> d)
{
    const RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.R_target)
        return;
    const int64_t R = c->R_cur;
    const double* W = d.cdf;
    double u;
    if (d.unif) {
        u = d.unif[k];
    } else {
        const u32x4 w = philox10((uint32_t)k, c->temp_index + 1u, 0u, kStreamMultinomial, d.key0, d.key1);
        u = uniform53(w.v[0], w.v[1]);
    }
    const double t = u * W[R - 1];
    // first j in [0, R) with W_j > t; R when there is none
    int64_t lo = 0, hi = R;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (W[mid] > t)
            hi = mid;
        else
            lo = mid + 1;
    }
    if (lo == R) {
        // t == W_{R-1}: the first j with W_j >= t
        lo = 0;
        hi = R - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (W[mid] >= t)
                hi = mid;
            else
                lo = mid + 1;
        }
    }
    atomicAdd(&d.counts[lo], 1);
}

// --------------------------------------------------------------------------
// PAMD step 2b: copy numbers, prefix sum, source of every destination slot
// --------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(kBlk) void k_counts(RunDev<real> d)
{
    __shared__ int64_t sh[kBlk];
    RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t R = c->R_cur;
    const double* E = d.epot[c->cur];
    const double db = c->dbeta, m = c->m, S = c->S;
    const double Rt = (double)d.R_target;
    const uint32_t ti = c->temp_index + 1u;
    const int64_t chunk = (R + kBlk - 1) / kBlk;
    const int64_t j0 = (int64_t)threadIdx.x * chunk;
    const int64_t j1 = (j0 + chunk < R) ? j0 + chunk : R;
    int64_t local = 0;
    if (d.resampling == PAMD_RESAMPLE_MULTINOMIAL) {
        // counts drawn by k_draw
        for (int64_t j = j0; j < j1; ++j)
            local += d.counts[j];
    } else if (d.resampling == PAMD_RESAMPLE_NONE) {
        for (int64_t j = j0; j < j1; ++j)
            d.counts[j] = 1;
        local = j1 > j0 ? j1 - j0 : 0;
    } else {
        for (int64_t j = j0; j < j1; ++j) {
            const double tau = Rt * exp(-db * (E[j] - m)) / S;
            const double fl = floor(tau);
            double u;
            if (d.unif) {
                u = d.unif[j];
            } else {
                const u32x4 w = philox10((uint32_t)j, ti, 0u, kStreamResample, d.key0, d.key1);
                u = uniform53(w.v[0], w.v[1]);
            }
            const int32_t cj = (int32_t)fl + ((u < tau - fl) ? 1 : 0);
            d.counts[j] = cj;
            local += cj;
        }
    }
    int64_t total = 0;
    int64_t off = block_exscan(local, sh, &total);
    if (total > d.R_cap || total <= 0) {
        if (threadIdx.x == 0) {
            c->R_new = total;
            atomicCAS(&c->error, 0, 3);
        }
        return;
    }
    for (int64_t j = j0; j < j1; ++j) {
        const int32_t cj = d.counts[j];
        for (int32_t q = 0; q < cj; ++q)
            d.src_of[off + q] = (int32_t)j;
        off += cj;
    }
    if (threadIdx.x == 0) {
        c->R_new = total;
        c->R_prev = R;
    }
}

// --------------------------------------------------------------------------
// PAMD step 2c: gather + velocity rescale + centre-of-mass recentring
// --------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(256) void k_gather(RunDev<real> d, double mtot)
{
    const RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t Rn = c->R_new;
    const int cur = c->cur;
    const real* src_all = d.slab[cur];
    real* dst_all = d.slab[cur ^ 1];
    const real vs = (real)sqrt(c->T_next / c->T_cur);
    const double ks = c->T_next / c->T_cur;   // kinetic energy of the rescaled copy
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int npad = d.npad, n = d.n;
    for (int64_t dd = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); dd < Rn; dd += nw) {
        const int32_t j = d.src_of[dd];
        const real* s = src_all + (size_t)j * 6 * npad;
        real* t = dst_all + (size_t)dd * 6 * npad;
        double mx = 0.0, my = 0.0, mz = 0.0;
        for (int a = lane; a < n; a += 64) {
            const double ma = d.mass[a];
            mx += ma * (double)s[a];
            my += ma * (double)s[npad + a];
            mz += ma * (double)s[2 * npad + a];
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            mx += __shfl_xor(mx, o);
            my += __shfl_xor(my, o);
            mz += __shfl_xor(mz, o);
        }
        const real cx = (real)(mx / mtot), cy = (real)(my / mtot), cz = (real)(mz / mtot);
        for (int a = lane; a < npad; a += 64) {
            if (a < n) {
                t[a] = s[a] - cx;
                t[npad + a] = s[npad + a] - cy;
                t[2 * npad + a] = s[2 * npad + a] - cz;
                t[3 * npad + a] = s[3 * npad + a] * vs;
                t[4 * npad + a] = s[4 * npad + a] * vs;
                t[5 * npad + a] = s[5 * npad + a] * vs;
            } else {
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    t[q * npad + a] = s[q * npad + a];
            }
        }
        if (lane == 0) {
            d.epot[cur ^ 1][dd] = d.epot[cur][j];
            d.ekin[cur ^ 1][dd] = d.ekin[cur][j] * ks;
            d.anc[cur ^ 1][dd] = d.anc[cur][j];
        }
    }
}

template <typename real>
__global__ void k_resample_finalize(RunDev<real> d)
{
    if (threadIdx.x != 0)
        return;
    RunCtl* c = d.ctl;
    if (c->error)
        return;
    c->cur ^= 1;
    c->R_cur = c->R_new;
    c->T_prev = c->T_cur;
    c->T_cur = c->T_next;
    c->temp_index += 1u;
    c->sum_lnQ += c->lnQ_last;
}

// Start of an MD call of one run: with a sticky error set (for instance a
// resampling over capacity) the MD, energy and finalize kernels of this call
// leave positions, velocities, energies and the step counter unchanged.
template <typename real>
__global__ void k_md_begin(RunDev<real> d)
{
    if (threadIdx.x == 0)
        d.ctl->frozen = d.ctl->error != 0;
}

template <typename real>
__global__ void k_md_finalize(RunDev<real> d, int n_steps)
{
    if (threadIdx.x != 0)
        return;
    if (!d.ctl->frozen)
        d.ctl->step += (uint32_t)n_steps;
    d.ctl->work = 0;
}

// --------------------------------------------------------------------------
// PAMD step 4: observables (population averages)
// --------------------------------------------------------------------------
struct ObsDev {   // mirrors pamd_obs
    double T, T_prev, lnQ_last, sum_lnQ, V_last, E_mean, E2_mean, K_mean, T_measured, Cv;
    int64_t R, families, temp_index, step;
    int32_t error, reserved;
};

template <typename real>
__global__ __launch_bounds__(kBlk) void k_observables(RunDev<real> d)
{
    __shared__ double sh[kBlk];
    const RunCtl* c = d.ctl;
    const int64_t R = c->R_cur;
    const int cur = c->cur;
    const double* E = d.epot[cur];
    double se = 0.0, se2 = 0.0, sk = 0.0;
    for (int64_t j = threadIdx.x; j < R; j += kBlk) {
        const double e = E[j];
        se += e;
        se2 += e * e;
        sk += d.ekin[cur][j];
    }
    se = block_sum(se, sh);
    se2 = block_sum(se2, sh);
    sk = block_sum(sk, sh);
    for (int64_t i = threadIdx.x; i < d.R_target; i += kBlk)
        d.fam[i] = 0;
    __syncthreads();
    for (int64_t j = threadIdx.x; j < R; j += kBlk) {
        const int32_t a = d.anc[cur][j];
        if (a >= 0 && a < d.R_target)
            d.fam[a] = 1;
    }
    __syncthreads();
    double nf = 0.0;
    for (int64_t i = threadIdx.x; i < d.R_target; i += kBlk)
        nf += (double)d.fam[i];
    nf = block_sum(nf, sh);
    if (threadIdx.x == 0) {
        ObsDev* o = reinterpret_cast<ObsDev*>(d.obs);
        const double Rd = (double)(R > 0 ? R : 1);
        o->T = c->T_cur;
        o->T_prev = c->T_prev;
        o->lnQ_last = c->lnQ_last;
        o->sum_lnQ = c->sum_lnQ;
        o->V_last = c->V_last;
        o->E_mean = se / Rd;
        o->E2_mean = se2 / Rd;
        o->K_mean = sk / Rd;
        o->T_measured = 2.0 * o->K_mean / (3.0 * d.n * d.kB);
        const double kT = d.kB * c->T_cur;
        o->Cv = (o->E2_mean - o->E_mean * o->E_mean) / (kT * kT);
        o->R = R;
        o->families = (int64_t)nf;
        o->temp_index = c->temp_index;
        o->step = c->step;
        o->error = c->error;
        o->reserved = 0;
    }
}

// --------------------------------------------------------------------------
// host-side launchers
// --------------------------------------------------------------------------
template <typename real>
hipError_t launch_init_t(const RunDev<real>& d, hipStream_t s)
{
    const int64_t total = d.R_target * (int64_t)d.npad;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_init<real>, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, d);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_resample_t(const RunDev<real>& d, double T_req, double mtot, int gather_blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_weights<real>, dim3(1), dim3(kBlk), 0, s, d, T_req);
    if (d.resampling == PAMD_RESAMPLE_MULTINOMIAL) {
        hipLaunchKernelGGL(k_cdf<real>, dim3(1), dim3(kBlk), 0, s, d);
        hipLaunchKernelGGL(k_draw<real>, dim3((unsigned)((d.R_target + 255) / 256)), dim3(256), 0, s, d);
    }
    hipLaunchKernelGGL(k_counts<real>, dim3(1), dim3(kBlk), 0, s, d);
    hipLaunchKernelGGL(k_gather<real>, dim3(gather_blocks), dim3(256), 0, s, d, mtot);
    hipLaunchKernelGGL(k_resample_finalize<real>, dim3(1), dim3(64), 0, s, d);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_md_begin_t(const RunDev<real>& d, hipStream_t s)
{
    hipLaunchKernelGGL(k_md_begin<real>, dim3(1), dim3(64), 0, s, d);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_md_finalize_t(const RunDev<real>& d, int n_steps, hipStream_t s)
{
    hipLaunchKernelGGL(k_md_finalize<real>, dim3(1), dim3(64), 0, s, d, n_steps);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_observables_t(const RunDev<real>& d, hipStream_t s)
{
    hipLaunchKernelGGL(k_observables<real>, dim3(1), dim3(kBlk), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_init(const RunDev<float>& d, hipStream_t s) { return launch_init_t(d, s); }
hipError_t launch_init(const RunDev<double>& d, hipStream_t s) { return launch_init_t(d, s); }
hipError_t launch_resample(const RunDev<float>& d, double T_req, double mtot, int gb, hipStream_t s)
{
    return launch_resample_t(d, T_req, mtot, gb, s);
}
hipError_t launch_resample(const RunDev<double>& d, double T_req, double mtot, int gb, hipStream_t s)
{
    return launch_resample_t(d, T_req, mtot, gb, s);
}
hipError_t launch_md_begin(const RunDev<float>& d, hipStream_t s) { return launch_md_begin_t(d, s); }
hipError_t launch_md_begin(const RunDev<double>& d, hipStream_t s) { return launch_md_begin_t(d, s); }
hipError_t launch_md_finalize(const RunDev<float>& d, int n, hipStream_t s) { return launch_md_finalize_t(d, n, s); }
hipError_t launch_md_finalize(const RunDev<double>& d, int n, hipStream_t s) { return launch_md_finalize_t(d, n, s); }
hipError_t launch_observables(const RunDev<float>& d, hipStream_t s) { return launch_observables_t(d, s); }
hipError_t launch_observables(const RunDev<double>& d, hipStream_t s) { return launch_observables_t(d, s); }

}  // namespace pamd
