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
// Every O(R) step runs over the whole GPU: blocks of 256 threads make
// per-block partial results and the block that finishes last (an atomic
// ticket) combines them in block order, so the FP64 sums have a fixed order
// and do not depend on scheduling.  The adaptive temperature takes a fixed
// sequence of such passes (a probe at the largest step, then Newton
// iterations that turn into no-ops once converged), so it replays from a HIP
// graph.  The gather is HBM bound: one wavefront per destination slab, 16-byte
// streaming accesses.
//
// Built with PAMD_BOUNDS_CHECK (the checked library variant), the scan and the
// gather verify every destination offset and source index and raise
// PAMD_ERR_INTERNAL instead of touching memory out of range.
#include <math.h>

#include "pamd.h"
#include "pamd_internal.h"
#include "philox.h"

namespace pamd {

constexpr int kRB = 256;             // threads per block of the multi-block passes
constexpr int kMaxPassBlocks = 256;  // blocks of a pass over the energies (<= kRB)
constexpr int kCdfT = 16;            // consecutive weights one thread sums (multinomial running sums)
constexpr int kWeightPasses = 6;     // adaptive step: Newton passes launched per resampling (typically 3-5 work)
constexpr int kMaxNewton = 64;       // Newton / bisection iterations before the step is taken as found

__host__ __device__ inline int pass_blocks(int64_t R_cap)
{
    const int64_t b = (R_cap + 4 * kRB - 1) / (4 * kRB);
    return b < 1 ? 1 : (b > kMaxPassBlocks ? kMaxPassBlocks : (int)b);
}
__host__ __device__ inline int64_t cdf_blocks(int64_t R_cap) { return (R_cap + kRB * kCdfT - 1) / (kRB * kCdfT); }
__host__ __device__ inline int64_t count_blocks(int64_t R_cap) { return (R_cap + kRB - 1) / kRB; }

// doubles of RunDev::part and int64 of RunDev::cpart for R_cap slots
size_t part_doubles(int64_t R_cap)
{
    const int64_t c = cdf_blocks(R_cap);
    return (size_t)(c > 8 * kMaxPassBlocks ? c : 8 * kMaxPassBlocks);
}
size_t cpart_count(int64_t R_cap) { return (size_t)count_blocks(R_cap); }

// ---------------------------------------------------------------------------
// block-level helpers (256 threads = 4 wavefronts)
// ---------------------------------------------------------------------------
// sums of N values over the block, returned to every thread (fixed order:
// butterfly within each wavefront, then the four wavefront sums)
template <int N, typename T>
__device__ __forceinline__ void block_sums(T (&v)[N], T* sh /* [N * 4] */)
{
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            v[k] += __shfl_xor(v[k], o);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < N; ++k)
            sh[4 * k + w] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k)
        v[k] = (sh[4 * k] + sh[4 * k + 1]) + (sh[4 * k + 2] + sh[4 * k + 3]);
    __syncthreads();
}

__device__ __forceinline__ double block_min(double v, double* sh /* [4] */)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        v = fmin(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = v;
    __syncthreads();
    v = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
    __syncthreads();
    return v;
}

// exclusive prefix sum over the block of one int per thread; *total = block sum
__device__ __forceinline__ int64_t block_exscan(int64_t v, int64_t* sh /* [kRB] */, int64_t* total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < kRB; o <<= 1) {
        const int64_t add = (t >= o) ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const int64_t inc = sh[t];
    *total = sh[kRB - 1];
    __syncthreads();
    return inc - v;
}

// True in every thread of the block that arrives last at this call; the
// partial results every other block wrote before its own call are visible to
// it afterwards.  The ticket is back at zero when the last block leaves.
__device__ __forceinline__ bool last_block(uint32_t* ticket, int* sflag)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        const int last = (t == gridDim.x - 1u);
        if (last)
            __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *sflag = last;
    }
    __syncthreads();
    const bool last = *sflag != 0;
    if (last)
        __threadfence();   // acquire: later loads see the other blocks' partials
    return last;
}

__device__ __forceinline__ void raise_error(RunCtl* c, int code) { atomicCAS(&c->error, 0, code); }

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
        c->ticket = 0;
        c->w_phase = 2;
        c->w_iter = 0;
        c->w_b = c->w_lo = c->w_hi = c->w_var = 0.0;
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
        d.fam[r] = 0;   // family flags start (and are left by every observables call) cleared
    }
}

// --------------------------------------------------------------------------
// PAMD step 2a: minimum, next temperature, normaliser
// --------------------------------------------------------------------------
// One update of the adaptive step from the weight moments at dbeta = c->w_b
// (S = sum w, S1 = sum w e, S2 = sum w^2, S21 = sum w^2 e, w = exp(-b e),
// e = E - m): phase 0 tests the largest step (to T_final) and starts Newton
// iterations from the Gaussian-energy estimate sqrt(ln(1 + V*) / var E);
// phase 1 is one safeguarded Newton step on V(b) = R S2 / S^2 - 1 = V*
// (dV/db = 2 R (S2 S1 / S^3 - S21 / S^2)), bisecting when the step leaves the
// bracket; converged (or after kMaxNewton iterations) it fixes T_next.
template <typename real>
__device__ void newton_update(const RunDev<real>& d, RunCtl* c, int64_t R, double S, double S1, double S2,
                              double S21)
{
    const double Rd = (double)R, Vt = d.V_target;
    const double V = Rd * S2 / (S * S) - 1.0;
    const double kB = d.kB, T = c->T_cur;
    if (c->w_phase == 0) {
        if (V <= Vt) {
            c->T_next = d.T_final;
            c->w_phase = 2;
            return;
        }
        const double lo = 0.0, hi = c->w_b;
        const double var = c->w_var;
        double b = var > 0.0 ? sqrt(log1p(Vt) / var) : 0.5 * hi;
        if (!(b > lo && b < hi))
            b = 0.5 * (lo + hi);
        c->w_lo = lo;
        c->w_hi = hi;
        c->w_b = b;
        c->w_phase = 1;
        return;
    }
    double b = c->w_b, lo = c->w_lo, hi = c->w_hi;
    if (V <= Vt)
        lo = b;
    else
        hi = b;
    const double dV = 2.0 * Rd * (S2 * S1 / (S * S * S) - S21 / (S * S));
    double bn = b - (V - Vt) / dV;
    if (!(bn > lo && bn < hi))
        bn = 0.5 * (lo + hi);
    const bool done = fabs(bn - b) <= 1e-13 * b || hi - lo <= 1e-12 * hi;
    c->w_lo = lo;
    c->w_hi = hi;
    c->w_b = bn;
    c->w_iter += 1;
    if (done || c->w_iter >= kMaxNewton) {
        c->T_next = 1.0 / (kB * (bn + 1.0 / (kB * T)));
        c->w_phase = 2;
    }
}

// pass 0: min E, non-finite check and the variance of E; for the adaptive
// choice also the weight sums at the largest step dmax (to T_final), each
// block relative to its own minimum and merged log-sum-exp style.  The last
// block fixes the next temperature when it is given (explicit or from the
// device schedule) or when the largest step is within the target variance,
// and starts the Newton iterations otherwise.
template <typename real>
__global__ __launch_bounds__(kRB) void k_w_stats(RunDev<real> d, double T_req)
{
    __shared__ double sh[4 * 3];
    __shared__ int sflag;
    RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t R = c->R_cur;
    const double* E = d.epot[c->cur];
    const double kB = d.kB, T = c->T_cur;
    const double dmax = 1.0 / (kB * d.T_final) - 1.0 / (kB * T);
    const bool probe = T_req == 0.0 && dmax > 0.0;
    const double e0 = E[0];   // shift against cancellation in the variance
    double mn = INFINITY;
    double v[3] = {0.0, 0.0, 0.0};   // sum (E - E_0), sum (E - E_0)^2, non-finite count
    const int64_t j0 = (int64_t)blockIdx.x * kRB + threadIdx.x, stride = (int64_t)gridDim.x * kRB;
    for (int64_t j = j0; j < R; j += stride) {
        const double e = E[j];
        if (!isfinite(e))
            v[2] += 1.0;
        mn = fmin(mn, e);
        v[0] += e - e0;
        v[1] += (e - e0) * (e - e0);
    }
    mn = block_min(mn, sh);
    block_sums<3>(v, sh);
    double p[2] = {0.0, 0.0};   // sum w, sum w^2 at dmax, w relative to this block's minimum
    if (probe && isfinite(mn)) {
        for (int64_t j = j0; j < R; j += stride) {
            const double w = exp(-dmax * (E[j] - mn));
            p[0] += w;
            p[1] += w * w;
        }
        block_sums<2>(p, sh);
    }
    double* part = d.part + 8 * (size_t)blockIdx.x;
    if (threadIdx.x == 0) {
        part[0] = mn;
        part[1] = v[0];
        part[2] = v[1];
        part[3] = v[2];
        part[4] = p[0];
        part[5] = p[1];
    }
    if (!last_block(&c->ticket, &sflag))
        return;
    // combine the block partials (fixed order)
    const int t = threadIdx.x;
    const bool have = t < (int)gridDim.x;
    const double* q = d.part + 8 * (size_t)t;
    double mb = have ? q[0] : INFINITY;
    mn = block_min(mb, sh);
    v[0] = have ? q[1] : 0.0;
    v[1] = have ? q[2] : 0.0;
    v[2] = have ? q[3] : 0.0;
    block_sums<3>(v, sh);
    if (v[2] > 0.0) {
        if (t == 0)
            raise_error(c, PAMD_ERR_NONFINITE);
        return;
    }
    if (probe) {
        // a block without elements has mb = inf and sums 0
        const double f = have && isfinite(mb) ? exp(-dmax * (mb - mn)) : 0.0;
        p[0] = have ? q[4] * f : 0.0;
        p[1] = have ? q[5] * f * f : 0.0;
        block_sums<2>(p, sh);
    }
    if (t != 0)
        return;
    const double Rd = (double)R;
    const double mean = v[0] / Rd;
    c->m = mn;
    c->w_var = v[1] / Rd - mean * mean;
    c->T_req = T_req;
    if (T_req > 0.0) {
        c->T_next = T_req;
        c->w_phase = 2;
    } else if (T_req < 0.0) {
        // device schedule: the next entry, or stay at the last one
        const int64_t nx = (int64_t)c->temp_index + 1;
        c->T_next = (d.sched && nx < d.n_sched) ? d.sched[nx] : T;
        c->w_phase = 2;
    } else if (!probe) {
        c->T_next = T;
        c->w_phase = 2;
    } else {
        c->w_b = dmax;
        c->w_phase = 0;
        c->w_iter = 0;
        newton_update(d, c, R, p[0], 0.0, p[1], 0.0);   // phase 0 reads V(dmax) from S and S2 only
    }
}

// weight moments of elements j = j0, j0 + stride, ... < R at dbeta b
__device__ __forceinline__ void moments(const double* E, int64_t R, int64_t j0, int64_t stride, double b, double m,
                                        double (&v)[4])
{
    for (int64_t j = j0; j < R; j += stride) {
        const double e = E[j] - m;
        const double w = exp(-b * e);
        const double ww = w * w;
        v[0] += w;
        v[1] += w * e;
        v[2] += ww;
        v[3] += ww * e;
    }
}

// one probe / Newton pass of the adaptive step (a no-op once T_next is
// fixed); the last pass of the sequence finishes an unconverged search in
// its last block alone
template <typename real>
__global__ __launch_bounds__(kRB) void k_w_pass(RunDev<real> d, int last_pass)
{
    __shared__ double sh[4 * 4];
    __shared__ int sflag;
    __shared__ int phase;
    RunCtl* c = d.ctl;
    if (c->error || c->w_phase == 2)
        return;
    const int64_t R = c->R_cur;
    const double* E = d.epot[c->cur];
    const double m = c->m;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    moments(E, R, (int64_t)blockIdx.x * kRB + threadIdx.x, (int64_t)gridDim.x * kRB, c->w_b, m, v);
    block_sums<4>(v, sh);
    if (threadIdx.x == 0) {
        double* part = d.part + 4 * (size_t)blockIdx.x;
        part[0] = v[0];
        part[1] = v[1];
        part[2] = v[2];
        part[3] = v[3];
    }
    if (!last_block(&c->ticket, &sflag))
        return;
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        v[k] = t < (int)gridDim.x ? d.part[4 * (size_t)t + k] : 0.0;
    block_sums<4>(v, sh);
    if (t == 0)
        newton_update(d, c, R, v[0], v[1], v[2], v[3]);
    __syncthreads();
    if (!last_pass)
        return;
    // rare: the search needs more iterations than the launched passes; every
    // iteration counts towards kMaxNewton, so the loop ends
    for (;;) {
        if (t == 0)
            phase = c->w_phase;
        __syncthreads();
        if (phase == 2)
            break;
        double u[4] = {0.0, 0.0, 0.0, 0.0};
        moments(E, R, t, kRB, c->w_b, m, u);
        block_sums<4>(u, sh);
        if (t == 0)
            newton_update(d, c, R, u[0], u[1], u[2], u[3]);
        __syncthreads();
    }
}

// S and S2 at the chosen step, ln Q, the weight variance
template <typename real>
__global__ __launch_bounds__(kRB) void k_w_final(RunDev<real> d)
{
    __shared__ double sh[4 * 2];
    __shared__ int sflag;
    RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t R = c->R_cur;
    const double* E = d.epot[c->cur];
    const double kB = d.kB;
    const double db = 1.0 / (kB * c->T_next) - 1.0 / (kB * c->T_cur);
    const double m = c->m;
    double v[2] = {0.0, 0.0};
    for (int64_t j = (int64_t)blockIdx.x * kRB + threadIdx.x; j < R; j += (int64_t)gridDim.x * kRB) {
        const double w = exp(-db * (E[j] - m));
        v[0] += w;
        v[1] += w * w;
    }
    block_sums<2>(v, sh);
    if (threadIdx.x == 0) {
        d.part[4 * (size_t)blockIdx.x] = v[0];
        d.part[4 * (size_t)blockIdx.x + 1] = v[1];
    }
    if (!last_block(&c->ticket, &sflag))
        return;
    const int t = threadIdx.x;
    v[0] = t < (int)gridDim.x ? d.part[4 * (size_t)t] : 0.0;
    v[1] = t < (int)gridDim.x ? d.part[4 * (size_t)t + 1] : 0.0;
    block_sums<2>(v, sh);
    if (t == 0) {
        const double S = v[0], S2 = v[1];
        c->dbeta = db;
        c->S = S;
        c->S2 = S2;
        c->lnQ_last = -db * m + log(S) - log((double)R);
        c->V_last = (double)R * S2 / (S * S) - 1.0;
    }
}

// --------------------------------------------------------------------------
// Multinomial resampling, running weight sums W_j = w_0 + ... + w_j in FP64:
// every thread sums kCdfT consecutive weights left to right; one thread per
// block scans the block's thread totals left to right, and (second kernel)
// the block totals in block order, W_j = off_block + (off_thread + partial_j)
// with every offset the rounded sum of the previous offset and total, so W
// never decreases (FP64 addition of non-negative values is monotone) and zero
// weights leave it flat.  Also clears the copy numbers.
// --------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(kRB) void k_cdf_a(RunDev<real> d)
{
    __shared__ double tot[kRB];
    const RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t R = c->R_cur;
    const double* E = d.epot[c->cur];
    const double db = c->dbeta, m = c->m;
    const int64_t j0 = ((int64_t)blockIdx.x * kRB + threadIdx.x) * kCdfT;
    double p[kCdfT];
    double run = 0.0;
#pragma unroll
    for (int i = 0; i < kCdfT; ++i) {
        const int64_t j = j0 + i;
        run += j < R ? exp(-db * (E[j] - m)) : 0.0;
        p[i] = run;
    }
    tot[threadIdx.x] = run;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int q = 0; q < kRB; ++q) {
            const double x = tot[q];
            tot[q] = acc;
            acc = acc + x;
        }
        d.part[blockIdx.x] = acc;
    }
    __syncthreads();
    const double toff = tot[threadIdx.x];
#pragma unroll
    for (int i = 0; i < kCdfT; ++i) {
        const int64_t j = j0 + i;
        if (j < R) {
            d.cdf[j] = toff + p[i];
            d.counts[j] = 0;
        }
    }
}

template <typename real>
__global__ __launch_bounds__(kRB) void k_cdf_b(RunDev<real> d)
{
    __shared__ double off;
    const RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t R = c->R_cur;
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int64_t q = 0; q < (int64_t)blockIdx.x; ++q)
            acc = acc + d.part[q];
        off = acc;
    }
    __syncthreads();
    const int64_t j0 = ((int64_t)blockIdx.x * kRB + threadIdx.x) * kCdfT;
#pragma unroll
    for (int i = 0; i < kCdfT; ++i) {
        const int64_t j = j0 + i;
        if (j < R)
            d.cdf[j] = off + d.cdf[j];
    }
}

// Multinomial resampling, the draws: one thread per draw k < R_target picks
// the first j with W_j > u_k W_{R-1} (if rounding leaves none, the first j
// with W_j >= u_k W_{R-1}) by binary search and adds one copy of j.
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
// PAMD step 2b: copy numbers (one thread per source slot), then the scan:
// every block takes its offset and the new population size from the block
// sums (exact integer sums), scans its own copy numbers and writes the source
// of every destination slot it owns
// --------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(kRB) void k_count_a(RunDev<real> d)
{
    __shared__ int64_t sh[4];
    const RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t R = c->R_cur;
    const int64_t j = (int64_t)blockIdx.x * kRB + threadIdx.x;
    int64_t cj = 0;
    if (j < R) {
        if (d.resampling == PAMD_RESAMPLE_MULTINOMIAL) {
            cj = d.counts[j];   // drawn by k_draw
        } else if (d.resampling == PAMD_RESAMPLE_NONE) {
            cj = 1;
            d.counts[j] = 1;
        } else {
            const double* E = d.epot[c->cur];
            const double tau = (double)d.R_target * exp(-c->dbeta * (E[j] - c->m)) / c->S;
            const double fl = floor(tau);
            double u;
            if (d.unif) {
                u = d.unif[j];
            } else {
                const u32x4 w = philox10((uint32_t)j, c->temp_index + 1u, 0u, kStreamResample, d.key0, d.key1);
                u = uniform53(w.v[0], w.v[1]);
            }
            cj = (int64_t)fl + ((u < tau - fl) ? 1 : 0);
            d.counts[j] = (int32_t)cj;
        }
    }
    int64_t v[1] = {cj};
    block_sums<1>(v, sh);
    if (threadIdx.x == 0)
        d.cpart[blockIdx.x] = v[0];
}

template <typename real>
__global__ __launch_bounds__(kRB) void k_count_b(RunDev<real> d)
{
    __shared__ int64_t sh[kRB];
    __shared__ int64_t sh4[8];
    RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t R = c->R_cur;
    int64_t v[2] = {0, 0};   // copies of the blocks before this one, all copies
    for (int64_t q = threadIdx.x; q < (int64_t)gridDim.x; q += kRB) {
        const int64_t x = d.cpart[q];
        v[1] += x;
        if (q < (int64_t)blockIdx.x)
            v[0] += x;
    }
    block_sums<2>(v, sh4);
    const int64_t total = v[1];
    if (total > d.R_cap || total <= 0) {
        // every block sees the same total: nothing is written
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            c->R_new = total;
            raise_error(c, PAMD_ERR_CAPACITY);
        }
        return;
    }
    const int64_t j = (int64_t)blockIdx.x * kRB + threadIdx.x;
    const int32_t cj = j < R ? d.counts[j] : 0;
    int64_t btot = 0;
    const int64_t off = v[0] + block_exscan(cj, sh, &btot);
#ifdef PAMD_BOUNDS_CHECK
    if (cj < 0 || off < 0 || off + cj > total) {
        raise_error(c, PAMD_ERR_INTERNAL);
        return;
    }
#endif
    for (int32_t q = 0; q < cj; ++q)
        d.src_of[off + q] = (int32_t)j;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->R_new = total;
        c->R_prev = R;
    }
}

// --------------------------------------------------------------------------
// PAMD step 2c: gather + velocity rescale + centre-of-mass recentring.  One
// wavefront per destination slot; the slab (6 arrays of npad reals) moves as
// 16-byte vectors, lane l holding vectors l, l + 64, ... (K per lane).
// --------------------------------------------------------------------------
template <typename real>
struct Vec16;
template <>
struct Vec16<float> {
    using T = float4;
    static constexpr int E = 4;
    __device__ static float get(const T& v, int e) { return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w; }
    __device__ static void set(T& v, int e, float x)
    {
        if (e == 0)
            v.x = x;
        else if (e == 1)
            v.y = x;
        else if (e == 2)
            v.z = x;
        else
            v.w = x;
    }
};
template <>
struct Vec16<double> {
    using T = double2;
    static constexpr int E = 2;
    __device__ static double get(const T& v, int e) { return e == 0 ? v.x : v.y; }
    __device__ static void set(T& v, int e, double x)
    {
        if (e == 0)
            v.x = x;
        else
            v.y = x;
    }
};

// 16-byte access of the gather: a native vector type for the streaming
// (non-temporal) loads and stores, each slab being read and written once
typedef uint32_t Nt16 __attribute__((ext_vector_type(4)));

template <typename real, int K>
__global__ __launch_bounds__(256) void k_gather(RunDev<real> d, double mtot)
{
    using VT = typename Vec16<real>::T;
    constexpr int E = Vec16<real>::E;
    RunCtl* c = d.ctl;
    if (c->error)
        return;
    const int64_t dd = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (dd >= c->R_new)
        return;
    const int lane = threadIdx.x & 63;
    const int cur = c->cur;
    const int npad = d.npad, n = d.n;
    const int32_t j = d.src_of[dd];
#ifdef PAMD_BOUNDS_CHECK
    if (j < 0 || (int64_t)j >= c->R_cur || dd >= d.R_cap) {
        if (lane == 0)
            raise_error(c, PAMD_ERR_INTERNAL);
        return;
    }
#endif
    const VT* src = reinterpret_cast<const VT*>(d.slab[cur] + (size_t)j * 6 * npad);
    VT* dst = reinterpret_cast<VT*>(d.slab[cur ^ 1] + (size_t)dd * 6 * npad);
    const int per = npad / E;           // vectors per coordinate array
    const int nv = 6 * per, npos = 3 * per;
    VT v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int q = lane + 64 * k;
        if (q < nv)
            v[k] = __builtin_bit_cast(VT, __builtin_nontemporal_load(reinterpret_cast<const Nt16*>(src) + q));
    }
    // mass-weighted centre of the source positions (FP64)
    double cm[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int q = lane + 64 * k;
        if (q < npos) {
            const int comp = q / per, a0 = (q - comp * per) * E;
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (a0 + e < n)
                    s += d.mass[a0 + e] * (double)Vec16<real>::get(v[k], e);
            cm[comp] += s;
        }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            cm[q] += __shfl_xor(cm[q], o);
    const real cx[3] = {(real)(cm[0] / mtot), (real)(cm[1] / mtot), (real)(cm[2] / mtot)};
    const real vs = (real)sqrt(c->T_next / c->T_cur);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int q = lane + 64 * k;
        if (q < nv) {
            const int comp = q / per, a0 = (q - comp * per) * E;
            VT o = v[k];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (a0 + e < n) {
                    const real x = Vec16<real>::get(o, e);
                    Vec16<real>::set(o, e, comp < 3 ? x - cx[comp] : x * vs);
                }
            }
            __builtin_nontemporal_store(__builtin_bit_cast(Nt16, o), reinterpret_cast<Nt16*>(dst) + q);
        }
    }
    if (lane == 0) {
        d.epot[cur ^ 1][dd] = d.epot[cur][j];
        d.ekin[cur ^ 1][dd] = d.ekin[cur][j] * (c->T_next / c->T_cur);   // kinetic energy of the rescaled copy
        d.anc[cur ^ 1][dd] = d.anc[cur][j];
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
// PAMD step 4: observables (population averages).  Pass a: sums of E, E^2
// and E_kin per block, family flags set; pass b (one thread per family
// flag): flags counted and cleared, the last block combines everything.
// --------------------------------------------------------------------------
struct ObsDev {   // mirrors pamd_obs
    double T, T_prev, lnQ_last, sum_lnQ, V_last, E_mean, E2_mean, K_mean, T_measured, Cv;
    int64_t R, families, temp_index, step;
    int32_t error, reserved;
};

template <typename real>
__global__ __launch_bounds__(kRB) void k_obs_a(RunDev<real> d)
{
    __shared__ double sh[4 * 3];
    const RunCtl* c = d.ctl;
    const int64_t R = c->R_cur;
    const int cur = c->cur;
    const double* E = d.epot[cur];
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t j = (int64_t)blockIdx.x * kRB + threadIdx.x; j < R; j += (int64_t)gridDim.x * kRB) {
        const double e = E[j];
        v[0] += e;
        v[1] += e * e;
        v[2] += d.ekin[cur][j];
        const int32_t a = d.anc[cur][j];
        if (a >= 0 && a < d.R_target)
            d.fam[a] = 1;
    }
    block_sums<3>(v, sh);
    if (threadIdx.x == 0) {
        double* part = d.part + 4 * (size_t)blockIdx.x;
        part[0] = v[0];
        part[1] = v[1];
        part[2] = v[2];
    }
}

template <typename real>
__global__ __launch_bounds__(kRB) void k_obs_b(RunDev<real> d, int a_blocks)
{
    __shared__ int64_t shi[4];
    __shared__ double sh[4 * 3];
    __shared__ int sflag;
    RunCtl* c = d.ctl;
    const int64_t i = (int64_t)blockIdx.x * kRB + threadIdx.x;
    int64_t f[1] = {0};
    if (i < d.R_target && d.fam[i]) {
        f[0] = 1;
        d.fam[i] = 0;
    }
    block_sums<1>(f, shi);
    if (threadIdx.x == 0)
        d.cpart[blockIdx.x] = f[0];
    if (!last_block(&c->ticket, &sflag))
        return;
    const int t = threadIdx.x;
    f[0] = 0;
    for (int64_t q = t; q < (int64_t)gridDim.x; q += kRB)
        f[0] += d.cpart[q];
    block_sums<1>(f, shi);
    double v[3] = {0.0, 0.0, 0.0};
    if (t < a_blocks) {
        const double* q = d.part + 4 * (size_t)t;
        v[0] = q[0];
        v[1] = q[1];
        v[2] = q[2];
    }
    block_sums<3>(v, sh);
    if (t == 0) {
        const int64_t R = c->R_cur;
        ObsDev* o = reinterpret_cast<ObsDev*>(d.obs);
        const double Rd = (double)(R > 0 ? R : 1);
        o->T = c->T_cur;
        o->T_prev = c->T_prev;
        o->lnQ_last = c->lnQ_last;
        o->sum_lnQ = c->sum_lnQ;
        o->V_last = c->V_last;
        o->E_mean = v[0] / Rd;
        o->E2_mean = v[1] / Rd;
        o->K_mean = v[2] / Rd;
        o->T_measured = 2.0 * o->K_mean / (3.0 * d.n * d.kB);
        const double kT = d.kB * c->T_cur;
        o->Cv = (o->E2_mean - o->E_mean * o->E_mean) / (kT * kT);
        o->R = R;
        o->families = f[0];
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

// 16-byte vectors per lane of the gather: ceil(6 npad / (16 / sizeof(real)) / 64), rounded up to 1, 2, 4, 8
template <typename real>
static hipError_t launch_gather(const RunDev<real>& d, double mtot, hipStream_t s)
{
    const int nv = 6 * d.npad / Vec16<real>::E;
    const int k = (nv + 63) / 64;
    const dim3 g((unsigned)((d.R_cap + 3) / 4)), b(256);
    if (k <= 1)
        hipLaunchKernelGGL((k_gather<real, 1>), g, b, 0, s, d, mtot);
    else if (k <= 2)
        hipLaunchKernelGGL((k_gather<real, 2>), g, b, 0, s, d, mtot);
    else if (k <= 4)
        hipLaunchKernelGGL((k_gather<real, 4>), g, b, 0, s, d, mtot);
    else
        hipLaunchKernelGGL((k_gather<real, 8>), g, b, 0, s, d, mtot);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_resample_t(const RunDev<real>& d, double T_req, double mtot, hipStream_t s)
{
    const int nbw = pass_blocks(d.R_cap);
    const unsigned nbc = (unsigned)count_blocks(d.R_cap);
    hipLaunchKernelGGL(k_w_stats<real>, dim3(nbw), dim3(kRB), 0, s, d, T_req);
    if (T_req == 0.0)
        for (int q = 0; q < kWeightPasses; ++q)
            hipLaunchKernelGGL(k_w_pass<real>, dim3(nbw), dim3(kRB), 0, s, d, q == kWeightPasses - 1 ? 1 : 0);
    hipLaunchKernelGGL(k_w_final<real>, dim3(nbw), dim3(kRB), 0, s, d);
    if (d.resampling == PAMD_RESAMPLE_MULTINOMIAL) {
        const unsigned nbf = (unsigned)cdf_blocks(d.R_cap);
        hipLaunchKernelGGL(k_cdf_a<real>, dim3(nbf), dim3(kRB), 0, s, d);
        hipLaunchKernelGGL(k_cdf_b<real>, dim3(nbf), dim3(kRB), 0, s, d);
        hipLaunchKernelGGL(k_draw<real>, dim3((unsigned)((d.R_target + 255) / 256)), dim3(256), 0, s, d);
    }
    hipLaunchKernelGGL(k_count_a<real>, dim3(nbc), dim3(kRB), 0, s, d);
    hipLaunchKernelGGL(k_count_b<real>, dim3(nbc), dim3(kRB), 0, s, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    e = launch_gather(d, mtot, s);
    if (e != hipSuccess)
        return e;
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
    const int nba = pass_blocks(d.R_cap);
    hipLaunchKernelGGL(k_obs_a<real>, dim3(nba), dim3(kRB), 0, s, d);
    hipLaunchKernelGGL(k_obs_b<real>, dim3((unsigned)count_blocks(d.R_target)), dim3(kRB), 0, s, d, nba);
    return hipGetLastError();
}

hipError_t launch_init(const RunDev<float>& d, hipStream_t s) { return launch_init_t(d, s); }
hipError_t launch_init(const RunDev<double>& d, hipStream_t s) { return launch_init_t(d, s); }
hipError_t launch_resample(const RunDev<float>& d, double T_req, double mtot, hipStream_t s)
{
    return launch_resample_t(d, T_req, mtot, s);
}
hipError_t launch_resample(const RunDev<double>& d, double T_req, double mtot, hipStream_t s)
{
    return launch_resample_t(d, T_req, mtot, s);
}
hipError_t launch_md_begin(const RunDev<float>& d, hipStream_t s) { return launch_md_begin_t(d, s); }
hipError_t launch_md_begin(const RunDev<double>& d, hipStream_t s) { return launch_md_begin_t(d, s); }
hipError_t launch_md_finalize(const RunDev<float>& d, int n, hipStream_t s) { return launch_md_finalize_t(d, n, s); }
hipError_t launch_md_finalize(const RunDev<double>& d, int n, hipStream_t s) { return launch_md_finalize_t(d, n, s); }
hipError_t launch_observables(const RunDev<float>& d, hipStream_t s) { return launch_observables_t(d, s); }
hipError_t launch_observables(const RunDev<double>& d, hipStream_t s) { return launch_observables_t(d, s); }

}  // namespace pamd
