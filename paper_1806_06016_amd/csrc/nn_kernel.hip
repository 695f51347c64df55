// Kernels of the learned multiple-time-step surrogate (an addition to the
// paper's method: it accelerates the MD update of PAMD step 3 by r-RESPA).
//
//   features   G[i, t, k] = sum over partners j of type t of
//              phi_k(r_ij) = exp(-(r_ij - mu_k)^2 / (2 s^2))  (VALU, one lane
//              per (configuration, atom) row, Gaussians by a multiplicative
//              recurrence in chunks of 8: one exponential per chunk and one
//              per pair)
//   MLP        E_i = w3 . silu(W2^T silu(W1^T G_i + b1) + b2) + b3 and its
//              input gradient dE_i/dG_i, fused in one kernel per 64-row tile
//              (BF16 MFMA 16x16x32, FP32 accumulate, activations in LDS)
//   forces     F_i = -sum_j (A_ij + A_ji) (x_i - x_j) / r_ij with
//              A_ij = sum_k dE_i/dG_i[t_j, k] phi_k'(r_ij)  (A staged in LDS)
//   training   the force-matching loss gradient: the directional derivative
//              v_i of the features along dL/dF (same kernel as the features),
//              then reverse mode through the forward-mode derivative of the
//              MLP (generic split-K BF16 MFMA GEMM + elementwise kernels),
//              Adam on FP32 master weights and the BF16 copies.
#include <stdint.h>

#include "nn_internal.h"

namespace pamd {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// float -> BF16, round to nearest even (one v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint32_t pack2(float a, float b)
{
    bf16x2 v;
    v[0] = (__bf16)a;
    v[1] = (__bf16)b;
    return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ void unpack8(const uint4& v, float* o)
{
    o[0] = __uint_as_float(v.x << 16);
    o[1] = __uint_as_float(v.x & 0xFFFF0000u);
    o[2] = __uint_as_float(v.y << 16);
    o[3] = __uint_as_float(v.y & 0xFFFF0000u);
    o[4] = __uint_as_float(v.z << 16);
    o[5] = __uint_as_float(v.z & 0xFFFF0000u);
    o[6] = __uint_as_float(v.w << 16);
    o[7] = __uint_as_float(v.w & 0xFFFF0000u);
}

// D (16x16) += A (16x32) B (32x16).  Lane l holds A[l % 16][8 (l / 16) + e],
// B[8 (l / 16) + e][l % 16] (e = 0..7) and D[4 (l / 16) + e][l % 16] (e = 0..3).
__device__ __forceinline__ f32x4 mfma(const uint4& a, const uint4& b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                     0, 0, 0);
}

__device__ __forceinline__ void silu_d(float h, float& a, float& d1)
{
    const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-h));
    a = h * sg;
    d1 = sg * (1.0f + h * (1.0f - sg));
}
__device__ __forceinline__ void silu_dd(float h, float& a, float& d1, float& d2)
{
    const float sg = 1.0f / (1.0f + __expf(-h));
    a = h * sg;
    d1 = sg * (1.0f + h * (1.0f - sg));
    d2 = sg * (1.0f - sg) * (2.0f + h * (1.0f - 2.0f * sg));
}

constexpr float kL2e = 1.44269504088896341f;   // log2(e)

// phi_k(r) = exp(-u_k^2 / 2), u_k = (r - mu_k) / s = u_0 - k, in chunks of 8:
//   phi_{k0+e} = P_e C_e,  P_0 = exp(-u_c^2 / 2),  P_{e+1} = P_e q,
//   q = exp(u_c),  C_e = exp(-e^2 / 2),  u_c = u_0 - k0.
// body(k, e, P_e) folds C_e into its multiply-add.  Each chunk restarts P_0
// from an exponential, so a chunk cannot underflow before its values matter;
// q comes from an exponential in the first chunk and from the previous
// chunk's q times exp(-8) after it (u_c falls by 8 per chunk).  u_0 >= -mu_0 / s
// > -40 for every distance, and u_c is clamped to 40: where it is, the
// chunk's values are below 1e-100, P_0 is 0 in FP32 and every q stays finite
// (below exp(40)); elsewhere q = exp(u_c) and the products stay finite
// (P_e <= exp(e^2 / 2) <= 4.4e10).
constexpr float kGauss[8] = {1.0f, 0.60653066f, 0.135335283f, 0.0111089965f,
                             0.000335462628f, 3.72665317e-06f, 1.52299797e-08f, 2.28973485e-11f};
constexpr float kExpM8 = 3.35462628e-04f;   // exp(-8)

template <typename Body>
__device__ __forceinline__ void rbf_chunks(float u0, Body&& body)
{
    float q = __builtin_amdgcn_exp2f(kL2e * fminf(fmaxf(u0, -40.f), 40.f));
#pragma unroll
    for (int ch = 0; ch < kRbf / 8; ++ch) {
        const float uc = fminf(fmaxf(u0 - (float)(8 * ch), -40.f), 40.f);
        float P = __builtin_amdgcn_exp2f(-0.5f * kL2e * uc * uc);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            body(8 * ch + e, e, P);
            P *= q;
        }
        q *= kExpM8;
    }
}

__device__ __forceinline__ int64_t io_count(const ConfIO& io) { return io.ctl ? io.ctl->R_cur : io.count; }
__device__ __forceinline__ const float* io_x(const ConfIO& io) { return io.ctl ? io.xbase[io.ctl->cur] : io.xbase[0]; }

// ---------------------------------------------------------------------------
// features (MODE 0) and their directional derivative along delta (MODE 1):
//   MODE 1: v_i[t, k] = sum_j phi_k'(r_ij) (x_i - x_j) . (delta_i - delta_j) / r_ij
// Block: floor(256 / n) configurations, one lane per (configuration, atom),
// atoms in the type-sorted order of Topo.  Output rows (c n + a) of 256 BF16
// values for atom a.
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_nn_feat(Topo tp, ConfIO io, const float* delta, uint16_t* out)
{
    __shared__ float sx[768];
    __shared__ float sd[MODE == 1 ? 768 : 1];
    const int n = tp.n;
    const int rpb = 256 / n;
    const int64_t count = io_count(io);
    const float* X = io_x(io);
    const int tid = threadIdx.x;
    const int rl = tid / n;
    const int i = tid - rl * n;          // sorted position of this lane's atom
    const bool on = rl < rpb;
    uint32_t ex0 = 0, ex1 = 0, ex2 = 0;
    int atom = 0;
    if (on) {
        ex0 = tp.excl[i][0];
        ex1 = tp.excl[i][1];
        ex2 = tp.excl[i][2];
        atom = tp.order[i];
    }
    const float inv_s = 1.0f / kSig;
    const float u_off = kMu0 / kSig;
    for (int64_t c0 = (int64_t)blockIdx.x * rpb; c0 < count; c0 += (int64_t)gridDim.x * rpb) {
        __syncthreads();
        {
            // rpb n 3 <= 768: three loads per thread, all in flight at once
            float v[3], dv[3];
#pragma unroll
            for (int it = 0; it < 3; ++it) {
                const int q = tid + 256 * it;
                const int cl = q / (3 * n);
                const int rem = q - cl * 3 * n;
                const int ps = rem / 3, comp = rem - 3 * ps;
                const int64_t c = c0 + cl;
                v[it] = dv[it] = 0.f;
                if (q < rpb * n * 3 && c < count) {
                    const int a = tp.order[ps];
                    v[it] = X[c * io.xs_conf + comp * io.xs_comp + a * io.xs_atom];
                    if constexpr (MODE == 1)
                        dv[it] = delta[(c * n + a) * 3 + comp];
                }
            }
#pragma unroll
            for (int it = 0; it < 3; ++it) {
                const int q = tid + 256 * it;
                if (q < rpb * n * 3) {
                    sx[q] = v[it];
                    if constexpr (MODE == 1)
                        sd[q] = dv[it];
                }
            }
        }
        __syncthreads();
        const int64_t c = c0 + rl;
        if (!on || c >= count)
            continue;
        const float* px = sx + rl * 3 * n;
        const float xi = px[3 * i], yi = px[3 * i + 1], zi = px[3 * i + 2];
        const float* pd = sd + (MODE == 1 ? rl * 3 * n : 0);
        float di0 = 0.f, di1 = 0.f, di2 = 0.f;
        if constexpr (MODE == 1) {
            di0 = pd[3 * i];
            di1 = pd[3 * i + 1];
            di2 = pd[3 * i + 2];
        }
        uint4* orow = reinterpret_cast<uint4*>(out + (size_t)(c * n + atom) * kFeat);
        for (int t = 0; t < kTypes; ++t) {
            float acc[kRbf];
#pragma unroll
            for (int k = 0; k < kRbf; ++k)
                acc[k] = 0.f;
#pragma unroll 2
            for (int j = tp.tstart[t]; j < tp.tstart[t + 1]; ++j) {
                const uint32_t word = j < 32 ? ex0 : (j < 64 ? ex1 : ex2);
                const bool excluded = (word >> (j & 31)) & 1u;
                const float dx = xi - px[3 * j], dy = yi - px[3 * j + 1], dz = zi - px[3 * j + 2];
                const float r2 = dx * dx + dy * dy + dz * dz;
                if constexpr (MODE == 0) {
                    // an excluded pair is moved far outside the basis (all values 0)
                    const float u0 = excluded ? 1e4f : __builtin_sqrtf(r2) * inv_s - u_off;
                    rbf_chunks(u0, [&](int k, int e, float P) { acc[k] = fmaf(P, kGauss[e], acc[k]); });
                } else {
                    const float rinv = excluded ? 0.f : __builtin_amdgcn_rsqf(r2);
                    const float w = (dx * (di0 - pd[3 * j]) + dy * (di1 - pd[3 * j + 1]) + dz * (di2 - pd[3 * j + 2])) *
                                    rinv;
                    const float u0 = r2 * rinv * inv_s - u_off;
                    const float cw = -w * inv_s;   // phi_k' = -(u_k / s) phi_k
                    rbf_chunks(u0, [&](int k, int e, float P) {
                        acc[k] = fmaf(P * kGauss[e], cw * (u0 - (float)k), acc[k]);
                    });
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint4 v;
                v.x = pack2(acc[8 * q], acc[8 * q + 1]);
                v.y = pack2(acc[8 * q + 2], acc[8 * q + 3]);
                v.z = pack2(acc[8 * q + 4], acc[8 * q + 5]);
                v.w = pack2(acc[8 * q + 6], acc[8 * q + 7]);
                orow[4 * t + q] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// fused MLP: per 64-row tile, energies e (FP32) and dE/dG (BF16).
// Four waves; layer outputs are split over the waves by column, activations
// pass through LDS (rows padded by 16 bytes against bank conflicts), weight
// fragments come from the (L2-resident) BF16 copies, kPf k-steps ahead of
// their use: one k-step's MFMAs take a small fraction of an L2 round trip.
// Every product is formed transposed (the weight fragment as the A operand),
// so a lane's four accumulator values are four adjacent columns of one row:
// bias and activation per column, one 8-byte LDS store per lane and tile, and
// the row energy summed over the four lane groups of the row.
// ---------------------------------------------------------------------------
constexpr int kTM = 64;
constexpr int kLdX = kFeat + 8;
constexpr int kLdH = kH + 8;
constexpr int kPf = 4;

// Weight fragments of k-steps [K0, K1) of the CT column tiles starting at
// output column c0 (WT: row = output column, ld elements, k contiguous).
template <int KS, int CT, int K0, int K1>
__device__ __forceinline__ void load_wfrag(uint4 (&b)[KS][CT], const uint16_t* WT, int ld, int c0, int l16, int g4)
{
    const uint16_t* p = WT + (size_t)(c0 + l16) * ld + 8 * g4;
#pragma unroll
    for (int ks = K0; ks < K1; ++ks)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
            b[ks][ct] = *reinterpret_cast<const uint4*>(p + (size_t)16 * ct * ld + 32 * ks);
}

// acc[rt][ct] = transposed tile (columns c0 + 16 ct + 4 g4 + e of row 16 rt + l16)
// of X W, X: 64 x 32 KS from LDS (row-major, ldx); the caller has loaded the
// fragments of the first kPf k-steps into b.
template <int KS, int CT>
__device__ __forceinline__ void layer_mfma(f32x4 (&acc)[4][CT], uint4 (&b)[KS][CT], const uint16_t* X, int ldx,
                                           const uint16_t* WT, int ld, int c0, int l16, int g4)
{
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
            acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t* p = WT + (size_t)(c0 + l16) * ld + 8 * g4;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        if (ks + kPf < KS) {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                b[ks + kPf < KS ? ks + kPf : ks][ct] =
                    *reinterpret_cast<const uint4*>(p + (size_t)16 * ct * ld + 32 * (ks + kPf));
        }
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            const uint4 a = *reinterpret_cast<const uint4*>(X + (16 * rt + l16) * ldx + 32 * ks + 8 * g4);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                acc[rt][ct] = mfma(b[ks][ct], a, acc[rt][ct]);
        }
    }
}

// four adjacent BF16 values, one 8-byte LDS store
__device__ __forceinline__ void st4(uint16_t* p, float a, float b, float c, float d)
{
    *reinterpret_cast<uint2*>(p) = uint2{pack2(a, b), pack2(c, d)};
}

__global__ __launch_bounds__(256, 3) void k_nn_mlp(Weights w, const uint16_t* G, uint16_t* gG, float* e_out,
                                                const RunCtl* ctl, int64_t rows_fixed, int n)
{
    // Xs: G tile, then (dead after layer 1) g2, then the dE/dG output tile;
    // Ys: a1, then g1.  52 KB in all: three workgroups per CU.
    __shared__ __align__(16) uint16_t Xs[kTM * kLdX];
    __shared__ __align__(16) uint16_t Ys[kTM * kLdH];
    __shared__ float es[4][kTM];
    uint16_t* Zs = Xs;
    const int64_t M = ctl ? ctl->R_cur * (int64_t)n : rows_fixed;
    const int64_t row0 = (int64_t)blockIdx.x * kTM;
    if (row0 >= M)
        return;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, l16 = lane & 15, g4 = lane >> 4;
    // this wave's output columns: 32 wave .. 32 wave + 31 of the hidden
    // layers, 64 wave .. 64 wave + 63 of dE/dG; c4: a lane's first column
    // within a 16-column tile
    const int c1 = 32 * wave, c4 = 4 * g4;

    uint4 b1f[kFeat / 32][2];
    load_wfrag<kFeat / 32, 2, 0, kPf>(b1f, w.W1T, kFeat, c1, l16, g4);
    {
        // all eight 16-byte loads of this thread in flight before the first LDS store
        uint4 v[kTM * 32 / 256];
#pragma unroll
        for (int it = 0; it < kTM * 32 / 256; ++it) {
            const int q = tid + 256 * it, r = q >> 5, ch = q & 31;
            v[it] = uint4{0u, 0u, 0u, 0u};
            if (row0 + r < M)
                v[it] = *reinterpret_cast<const uint4*>(G + (size_t)(row0 + r) * kFeat + ch * 8);
        }
#pragma unroll
        for (int it = 0; it < kTM * 32 / 256; ++it) {
            const int q = tid + 256 * it, r = q >> 5, ch = q & 31;
            *reinterpret_cast<uint4*>(Xs + r * kLdX + ch * 8) = v[it];
        }
    }
    __syncthreads();

    // layer 1: h1 = G W1 + b1; a1 = silu(h1) to Ys, s1 = silu'(h1) kept
    float s1[4][2][4];
    uint4 b2f[kH / 32][2];
    {
        f32x4 acc[4][2];
        layer_mfma<kFeat / 32, 2>(acc, b1f, Xs, kLdX, w.W1T, kFeat, c1, l16, g4);
        load_wfrag<kH / 32, 2, 0, kPf>(b2f, w.W2T, kH, c1, l16, g4);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int col = c1 + 16 * ct + c4;
            float bias[4], a1[4];
#pragma unroll
            for (int e = 0; e < 4; ++e)
                bias[e] = w.b1[col + e];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    silu_d(acc[rt][ct][e] + bias[e], a1[e], s1[rt][ct][e]);
                st4(Ys + (16 * rt + l16) * kLdH + col, a1[0], a1[1], a1[2], a1[3]);
            }
        }
    }
    __syncthreads();

    // layer 2: h2 = a1 W2 + b2; e partial = a2 . w3; g2 = w3 silu'(h2) to Zs
    uint4 b3f[kH / 32][2];
    {
        f32x4 acc[4][2];
        layer_mfma<kH / 32, 2>(acc, b2f, Ys, kLdH, w.W2T, kH, c1, l16, g4);
        load_wfrag<kH / 32, 2, 0, kPf>(b3f, w.W2, kH, c1, l16, g4);
        float ep[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int col = c1 + 16 * ct + c4;
            float bias[4], w3c[4], g2[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                bias[e] = w.b2[col + e];
                w3c[e] = w.w3[col + e];
            }
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float a2, s2;
                    silu_d(acc[rt][ct][e] + bias[e], a2, s2);
                    ep[rt] = fmaf(a2, w3c[e], ep[rt]);
                    g2[e] = w3c[e] * s2;
                }
                st4(Zs + (16 * rt + l16) * kLdH + col, g2[0], g2[1], g2[2], g2[3]);
            }
        }
        // the row's 32 columns of this wave sit in the four lane groups
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            float v = ep[rt];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (g4 == 0)
                es[wave][16 * rt + l16] = v;
        }
    }
    __syncthreads();

    // g1 = (g2 W2^T) * silu'(h1): the same columns as this wave's layer-1 output
    const int c2 = 64 * wave;
    uint4 b4f[kH / 32][4];
    {
        f32x4 acc[4][2];
        layer_mfma<kH / 32, 2>(acc, b3f, Zs, kLdH, w.W2, kH, c1, l16, g4);
        load_wfrag<kH / 32, 4, 0, kPf>(b4f, w.W1, kH, c2, l16, g4);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int col = c1 + 16 * ct + c4;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
                st4(Ys + (16 * rt + l16) * kLdH + col, acc[rt][ct][0] * s1[rt][ct][0], acc[rt][ct][1] * s1[rt][ct][1],
                    acc[rt][ct][2] * s1[rt][ct][2], acc[rt][ct][3] * s1[rt][ct][3]);
        }
    }
    __syncthreads();

    // dE/dG = g1 W1^T: this wave's columns 64 wave .. 64 wave + 63, staged in Xs
    {
        f32x4 acc[4][4];
        layer_mfma<kH / 32, 4>(acc, b4f, Ys, kLdH, w.W1, kH, c2, l16, g4);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int col = c2 + 16 * ct + c4;
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
                st4(Xs + (16 * rt + l16) * kLdX + col, acc[rt][ct][0], acc[rt][ct][1], acc[rt][ct][2],
                    acc[rt][ct][3]);
        }
    }
    __syncthreads();
    for (int q = tid; q < kTM * 32; q += 256) {
        const int r = q >> 5, ch = q & 31;
        if (row0 + r < M)
            *reinterpret_cast<uint4*>(gG + (size_t)(row0 + r) * kFeat + ch * 8) =
                *reinterpret_cast<const uint4*>(Xs + r * kLdX + ch * 8);
    }
    if (tid < kTM && row0 + tid < M)
        e_out[row0 + tid] = es[0][tid] + es[1][tid] + es[2][tid] + es[3][tid] + w.b3[0];
}

// ---------------------------------------------------------------------------
// forces from dE/dG (and, optionally, configuration energies from the row
// energies).  Pass 1: lane (c, i) fills A[c][i][j] = dE_i / dr_ij for every j;
// pass 2: F_i = -sum_j (A_ij + A_ji) (x_i - x_j) / r_ij.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_nn_force(Topo tp, ConfIO io, const uint16_t* gG, const float* e_row,
                                                  float* E_out)
{
    extern __shared__ __align__(16) float fsm[];
    const int n = tp.n;
    const int rpb = 256 / n;
    float* sx = fsm;                  // [rpb][n][3]
    float* A = sx + rpb * n * 3;      // [rpb][n][n]
    float* es = A + rpb * n * n;      // [256]
    const int64_t count = io_count(io);
    const float* X = io_x(io);
    const int tid = threadIdx.x;
    const int rl = tid / n;
    const int i = tid - rl * n;          // sorted position of this lane's atom
    const bool on = rl < rpb;
    uint32_t ex0 = 0, ex1 = 0, ex2 = 0;
    int atom = 0;
    if (on) {
        ex0 = tp.excl[i][0];
        ex1 = tp.excl[i][1];
        ex2 = tp.excl[i][2];
        atom = tp.order[i];
    }
    const float inv_s = 1.0f / kSig;
    const float u_off = kMu0 / kSig;
    for (int64_t c0 = (int64_t)blockIdx.x * rpb; c0 < count; c0 += (int64_t)gridDim.x * rpb) {
        __syncthreads();
        {
            float v[3];
#pragma unroll
            for (int it = 0; it < 3; ++it) {
                const int q = tid + 256 * it;
                const int cl = q / (3 * n);
                const int rem = q - cl * 3 * n;
                const int ps = rem / 3, comp = rem - 3 * ps;
                const int64_t c = c0 + cl;
                v[it] = (q < rpb * n * 3 && c < count)
                            ? X[c * io.xs_conf + comp * io.xs_comp + tp.order[ps] * io.xs_atom]
                            : 0.f;
            }
#pragma unroll
            for (int it = 0; it < 3; ++it)
                if (tid + 256 * it < rpb * n * 3)
                    sx[tid + 256 * it] = v[it];
        }
        __syncthreads();
        const int64_t c = c0 + rl;
        const bool act = on && c < count;
        const float* px = sx + rl * 3 * n;
        float xi = 0.f, yi = 0.f, zi = 0.f;
        if (act) {
            xi = px[3 * i];
            yi = px[3 * i + 1];
            zi = px[3 * i + 2];
            const uint4* grow = reinterpret_cast<const uint4*>(gG + (size_t)(c * n + atom) * kFeat);
            float* Ai = A + (rl * n + i) * n;
            // the 64-byte segment of the next type is loaded while this one is used
            uint4 nxt[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                nxt[q] = grow[q];
            for (int t = 0; t < kTypes; ++t) {
                uint4 cur[4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    cur[q] = nxt[q];
                if (t + 1 < kTypes) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        nxt[q] = grow[4 * (t + 1) + q];
                }
                if (tp.tstart[t] == tp.tstart[t + 1])
                    continue;
                // c0[k] = dE/dG[t, k] C_e, c1[k] = k c0[k]:
                //   dE_i/dr_ij = -(1/s) sum_k dE/dG[t, k] phi_k (u_0 - k) = -(1/s) (u_0 S0 - S1)
                float c0[kRbf], c1[kRbf];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    unpack8(cur[q], c0 + 8 * q);
#pragma unroll
                for (int k = 0; k < kRbf; ++k) {
                    c0[k] *= kGauss[k & 7];
                    c1[k] = c0[k] * (float)k;
                }
#pragma unroll 2
                for (int j = tp.tstart[t]; j < tp.tstart[t + 1]; ++j) {
                    const uint32_t word = j < 32 ? ex0 : (j < 64 ? ex1 : ex2);
                    const bool excluded = (word >> (j & 31)) & 1u;
                    const float dx = xi - px[3 * j], dy = yi - px[3 * j + 1], dz = zi - px[3 * j + 2];
                    const float u0 = excluded ? 1e4f : __builtin_sqrtf(dx * dx + dy * dy + dz * dz) * inv_s - u_off;
                    float S0 = 0.f, S1 = 0.f;
                    rbf_chunks(u0, [&](int k, int e, float P) {
                        S0 = fmaf(P, c0[k], S0);
                        S1 = fmaf(P, c1[k], S1);
                    });
                    Ai[j] = excluded ? 0.f : -inv_s * (u0 * S0 - S1);
                }
            }
        }
        __syncthreads();
        float eacc = 0.f;
        if (act) {
            const float* Ai = A + (rl * n + i) * n;
            const float* Ab = A + rl * n * n;
            float fx = 0.f, fy = 0.f, fz = 0.f;
            for (int j = 0; j < n; ++j) {
                const float s = Ai[j] + Ab[j * n + i];
                const float dx = xi - px[3 * j], dy = yi - px[3 * j + 1], dz = zi - px[3 * j + 2];
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float g = (j == i) ? 0.f : s * __builtin_amdgcn_rsqf(r2);
                fx -= g * dx;
                fy -= g * dy;
                fz -= g * dz;
            }
            float* f = io.fout + c * io.fs_conf + atom * io.fs_atom;
            f[0] = fx;
            f[io.fs_comp] = fy;
            f[2 * io.fs_comp] = fz;
            if (E_out)
                eacc = e_row[c * n + atom];
        }
        if (E_out) {
            es[tid] = eacc;
            __syncthreads();
            if (act && i == 0) {
                float s = 0.f;
                for (int a = 0; a < n; ++a)
                    s += es[rl * n + a];
                E_out[c] = s;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// training: generic BF16 GEMM with FP32 output, split over K by blockIdx.z
//   C_z[m][n] = sum_{k in chunk z} A(m, k) B(k, n),
//   A(m, k) = A[m sam + k sak],  B(k, n) = B[k sbk + n sbn]
// 64x64 tiles, four waves of 32x32, operands staged k-contiguous in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gemm(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B,
                                              int64_t sbk, int64_t sbn, float* C, int64_t M, int64_t N, int64_t K,
                                              int64_t kchunk)
{
    __shared__ __align__(16) uint16_t As[64 * 40];
    __shared__ __align__(16) uint16_t Bs[64 * 40];
    const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
    const int64_t kb = (int64_t)blockIdx.z * kchunk;
    const int64_t ke = (K < kb + kchunk) ? K : kb + kchunk;
    C += (size_t)blockIdx.z * M * N;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, l16 = lane & 15, g4 = lane >> 4;
    const int wm = wave >> 1, wn = wave & 1;
    f32x4 acc[2][2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
            acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int sr = tid >> 2, sk = (tid & 3) * 8;
    for (int64_t k0 = kb; k0 < ke; k0 += 32) {
        __syncthreads();
        {
            uint16_t va[8], vb[8];
            const int64_t m = m0 + sr, nn = n0 + sr;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t k = k0 + sk + e;
                va[e] = (m < M && k < ke) ? A[m * sam + k * sak] : (uint16_t)0;
                vb[e] = (nn < N && k < ke) ? B[k * sbk + nn * sbn] : (uint16_t)0;
            }
            uint4 pa, pb;
            pa.x = va[0] | ((uint32_t)va[1] << 16);
            pa.y = va[2] | ((uint32_t)va[3] << 16);
            pa.z = va[4] | ((uint32_t)va[5] << 16);
            pa.w = va[6] | ((uint32_t)va[7] << 16);
            pb.x = vb[0] | ((uint32_t)vb[1] << 16);
            pb.y = vb[2] | ((uint32_t)vb[3] << 16);
            pb.z = vb[4] | ((uint32_t)vb[5] << 16);
            pb.w = vb[6] | ((uint32_t)vb[7] << 16);
            *reinterpret_cast<uint4*>(As + sr * 40 + sk) = pa;
            *reinterpret_cast<uint4*>(Bs + sr * 40 + sk) = pb;
        }
        __syncthreads();
        uint4 a[2], b[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
            a[rt] = *reinterpret_cast<const uint4*>(As + (32 * wm + 16 * rt + l16) * 40 + 8 * g4);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
            b[ct] = *reinterpret_cast<const uint4*>(Bs + (32 * wn + 16 * ct + l16) * 40 + 8 * g4);
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
                acc[rt][ct] = mfma(a[rt], b[ct], acc[rt][ct]);
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = m0 + 32 * wm + 16 * rt + 4 * g4 + e;
                const int64_t col = n0 + 32 * wn + 16 * ct + l16;
                if (row < M && col < N)
                    C[row * N + col] = acc[rt][ct][e];
            }
}

// out[i] = alpha * sum_z part[z len + i]
__global__ void k_reduce(const float* part, int nz, int64_t len, float alpha, float* out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < nz; ++z)
            s += part[(size_t)z * len + i];
        out[i] = alpha * s;
    }
}

// partial column sums of X [M][128]: part[b][col] over the rows of block b
__global__ __launch_bounds__(256) void k_colsum(const float* X, int64_t M, float* part)
{
    __shared__ float sh[256];
    const int col = threadIdx.x & (kH - 1), half = threadIdx.x >> 7;
    const int64_t per = (M + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = (r0 + per < M) ? r0 + per : M;
    float s = 0.f;
    for (int64_t r = r0 + half; r < r1; r += 2)
        s += X[r * kH + col];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (half == 0)
        part[(size_t)blockIdx.x * kH + col] = sh[col] + sh[col + kH];
}

// after [h1 | dh1] = [G ; V] W1 (rows 0..M-1 and M..2M-1 of HD)
__global__ void k_tr_e1(int64_t M, const float* HD, const float* b1, uint16_t* AD, float* S1, float* T1)
{
    const int64_t len = M * kH;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < len; q += (int64_t)gridDim.x * blockDim.x) {
        const int col = (int)(q & (kH - 1));
        float a, d1, d2;
        silu_dd(HD[q] + b1[col], a, d1, d2);
        const float dh = HD[len + q];
        AD[q] = (uint16_t)bf16_bits(a);            // a1
        AD[len + q] = (uint16_t)bf16_bits(d1 * dh); // da1
        S1[q] = d1;
        T1[q] = d2 * dh;
    }
}

// after [h2 | dh2] = [a1 ; da1] W2: adjoints of the directional derivative
//   rows 0..M-1:  hbar2 = w3 silu''(h2) dh2,  rows M..2M-1:  dhdot2 = w3 silu'(h2)
__global__ void k_tr_e2(int64_t M, const float* HD, const float* b2, const float* w3, uint16_t* D2, float* HB2,
                        float* DA2)
{
    const int64_t len = M * kH;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < len; q += (int64_t)gridDim.x * blockDim.x) {
        const int col = (int)(q & (kH - 1));
        float a, d1, d2;
        silu_dd(HD[q] + b2[col], a, d1, d2);
        const float dh = HD[len + q];
        const float hb = w3[col] * d2 * dh;
        D2[q] = (uint16_t)bf16_bits(hb);
        D2[len + q] = (uint16_t)bf16_bits(w3[col] * d1);
        HB2[q] = hb;
        DA2[q] = d1 * dh;
    }
}

// after [abar1 | dadot1] = [hbar2 ; dhdot2] W2^T
//   rows 0..M-1:  hbar1 = abar1 silu'(h1) + dadot1 silu''(h1) dh1,  rows M..:  dhdot1 = dadot1 silu'(h1)
__global__ void k_tr_e3(int64_t M, const float* AB, const float* S1, const float* T1, uint16_t* D1, float* HB1)
{
    const int64_t len = M * kH;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < len; q += (int64_t)gridDim.x * blockDim.x) {
        const float ab = AB[q], dd = AB[len + q];
        const float hb = ab * S1[q] + dd * T1[q];
        D1[q] = (uint16_t)bf16_bits(hb);
        D1[len + q] = (uint16_t)bf16_bits(dd * S1[q]);
        HB1[q] = hb;
    }
}

// force-matching loss: delta = dL/dF = 2 (F - F*) / len, part[b] = block sum of (F - F*)^2 / len
__global__ __launch_bounds__(256) void k_nn_loss(const float* F, const float* Ft, int64_t len, float* delta,
                                                 float* part)
{
    __shared__ float sh[256];
    const float inv = 1.0f / (float)len;
    float s = 0.f;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < len; q += (int64_t)gridDim.x * blockDim.x) {
        const float d = F[q] - Ft[q];
        delta[q] = 2.0f * d * inv;
        s += d * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = sh[0] * inv;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (__builtin_sqrtf(vi / bc2) + eps);
}

// BF16 copies of W1, W2 and their transposes from the FP32 master vector
__global__ void k_nn_refresh(const float* p, uint16_t* W1, uint16_t* W1T, uint16_t* W2, uint16_t* W2T)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < kFeat * kH) {
        const int f = q / kH, h = q - f * kH;
        const uint16_t b = (uint16_t)bf16_bits(p[oW1 + q]);
        W1[q] = b;
        W1T[h * kFeat + f] = b;
    }
    if (q < kH * kH) {
        const int a = q / kH, c = q - a * kH;
        const uint16_t b = (uint16_t)bf16_bits(p[oW2 + q]);
        W2[q] = b;
        W2T[c * kH + a] = b;
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static int grid_of(int64_t work, int per_block, int cap)
{
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1)
        g = 1;
    return (int)(g < cap ? g : cap);
}

size_t force_lds_bytes(int n)
{
    const int rpb = 256 / n;
    return (size_t)(rpb * n * 3 + rpb * n * n + 256) * sizeof(float);
}

hipError_t nn_setup()
{
    static bool done = false;
    if (done)
        return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)k_nn_force, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)force_lds_bytes(kMaxN));
    if (e == hipSuccess)
        done = true;
    return e;
}

hipError_t launch_features(const Topo& tp, const ConfIO& io, int64_t count_max, const float* delta, uint16_t* out,
                           hipStream_t s)
{
    const int rpb = 256 / tp.n;
    const int grid = grid_of(count_max, rpb, 1 << 20);
    if (delta)
        hipLaunchKernelGGL(k_nn_feat<1>, dim3(grid), dim3(256), 0, s, tp, io, delta, out);
    else
        hipLaunchKernelGGL(k_nn_feat<0>, dim3(grid), dim3(256), 0, s, tp, io, delta, out);
    return hipGetLastError();
}

hipError_t launch_mlp(const Weights& w, const uint16_t* G, uint16_t* gG, float* e, const RunCtl* ctl,
                      int64_t rows_max, int n, hipStream_t s)
{
    const int grid = grid_of(rows_max, kTM, 1 << 30);
    hipLaunchKernelGGL(k_nn_mlp, dim3(grid), dim3(256), 0, s, w, G, gG, e, ctl, rows_max, n);
    return hipGetLastError();
}

hipError_t launch_force(const Topo& tp, const ConfIO& io, int64_t count_max, const uint16_t* gG, const float* e_row,
                        float* E_out, hipStream_t s)
{
    hipError_t e = nn_setup();
    if (e != hipSuccess)
        return e;
    const int rpb = 256 / tp.n;
    const int grid = grid_of(count_max, rpb, 1 << 20);
    hipLaunchKernelGGL(k_nn_force, dim3(grid), dim3(256), force_lds_bytes(tp.n), s, tp, io, gG, e_row, E_out);
    return hipGetLastError();
}

hipError_t launch_gemm(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk, int64_t sbn,
                       float* C, int64_t M, int64_t N, int64_t K, int nz, hipStream_t s)
{
    int64_t kchunk = (K + nz - 1) / nz;
    kchunk = (kchunk + 31) / 32 * 32;
    const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)nz);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C, M, N, K, kchunk);
    return hipGetLastError();
}

hipError_t launch_reduce(const float* part, int nz, int64_t len, float alpha, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(grid_of(len, 256, 4096)), dim3(256), 0, s, part, nz, len, alpha, out);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* X, int64_t M, float* part, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_colsum, dim3(nb), dim3(256), 0, s, X, M, part);
    return hipGetLastError();
}

hipError_t launch_train_e1(int64_t M, const float* HD, const float* b1, uint16_t* AD, float* S1, float* T1,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_tr_e1, dim3(grid_of(M * kH, 256, 8192)), dim3(256), 0, s, M, HD, b1, AD, S1, T1);
    return hipGetLastError();
}
hipError_t launch_train_e2(int64_t M, const float* HD, const float* b2, const float* w3, uint16_t* D2, float* HB2,
                           float* DA2, hipStream_t s)
{
    hipLaunchKernelGGL(k_tr_e2, dim3(grid_of(M * kH, 256, 8192)), dim3(256), 0, s, M, HD, b2, w3, D2, HB2, DA2);
    return hipGetLastError();
}
hipError_t launch_train_e3(int64_t M, const float* AB, const float* S1, const float* T1, uint16_t* D1, float* HB1,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_tr_e3, dim3(grid_of(M * kH, 256, 8192)), dim3(256), 0, s, M, AB, S1, T1, D1, HB1);
    return hipGetLastError();
}

hipError_t launch_loss(const float* F, const float* Ft, int64_t len, float* delta, float* part, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_nn_loss, dim3(nb), dim3(256), 0, s, F, Ft, len, delta, part);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_refresh(const float* p, uint16_t* W1, uint16_t* W1T, uint16_t* W2, uint16_t* W2T, hipStream_t s)
{
    hipLaunchKernelGGL(k_nn_refresh, dim3((kFeat * kH + 255) / 256), dim3(256), 0, s, p, W1, W1T, W2, W2T);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace pamd
