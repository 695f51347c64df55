// Internal structures of the learned multiple-time-step surrogate: a per-atom
// MLP on Gaussian radial features whose forces replace the nonbonded force
// inside the short r-RESPA steps.  Shared by nn_kernel.hip, the RESPA kernel
// of md_kernel.hip and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "pamd_internal.h"

namespace pamd {
namespace nn {

constexpr int kTypes = 8;                 // atom types of the feature channels
constexpr int kRbf = 32;                  // Gaussians per type
constexpr int kFeat = kTypes * kRbf;      // 256 inputs per atom
constexpr int kH = 128;                   // both hidden widths
constexpr int kMaxN = 80;
// flat FP32 parameter vector: W1 [256][128], b1 [128], W2 [128][128], b2 [128], w3 [128], b3
constexpr int oW1 = 0;
constexpr int ob1 = oW1 + kFeat * kH;
constexpr int oW2 = ob1 + kH;
constexpr int ob2 = oW2 + kH * kH;
constexpr int ow3 = ob2 + kH;
constexpr int ob3 = ow3 + kH;
constexpr int kParams = ob3 + 1;

// Gaussian centres mu_k = kMu0 + k * kSig (nm), common width kSig
constexpr float kMu0 = 0.1f;
constexpr float kSig = 1.1f / 31.0f;

// the molecule as the surrogate sees it (passed by value)
// Kernels work in "sorted" atom order: position p holds atom order[p], atoms
// sorted by type, so the partners of type t are the contiguous positions
// tstart[t] .. tstart[t + 1] - 1.
struct Topo {
    int32_t n;
    int32_t tstart[kTypes + 1];
    uint8_t order[kMaxN];         // atom at sorted position p
    uint8_t atype[kMaxN];         // type of atom a (natural order)
    uint32_t excl[kMaxN][3];      // bit q of position p: the pair (order[p], order[q]) carries no
                                  // feature (self, 1-2, 1-3)
};

// BF16 weight copies (row-major) and FP32 vectors used by the kernels
struct Weights {
    const uint16_t* W1T;   // [128][256]  W1 transposed (forward B operand, k contiguous)
    const uint16_t* W1;    // [256][128]  (input-gradient B operand)
    const uint16_t* W2T;   // [128][128]  W2 transposed
    const uint16_t* W2;    // [128][128]
    const float* b1;       // [128]
    const float* b2;       // [128]
    const float* w3;       // [128]
    const float* b3;       // [1]
};

// where configurations come from and where forces go.  Slab mode (ctl set):
// the population of one MD run, count = ctl->R_cur, positions in
// xbase[ctl->cur]; array mode: `count` configurations at xbase[0].
struct ConfIO {
    const float* xbase[2];
    float* fout;
    const RunCtl* ctl;
    int64_t count;
    int64_t xs_conf, xs_comp, xs_atom;   // position strides (elements)
    int64_t fs_conf, fs_comp, fs_atom;   // force strides
};

// kernel launchers (nn_kernel.hip)
hipError_t launch_features(const Topo& tp, const ConfIO& io, int64_t count_max, const float* delta, uint16_t* out,
                           hipStream_t s);
hipError_t launch_mlp(const Weights& w, const uint16_t* G, uint16_t* gG, float* e, const RunCtl* ctl,
                      int64_t rows_max, int n, hipStream_t s);
hipError_t launch_force(const Topo& tp, const ConfIO& io, int64_t count_max, const uint16_t* gG, const float* e_row,
                        float* E_out, hipStream_t s);
hipError_t launch_gemm(const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B, int64_t sbk, int64_t sbn,
                       float* C, int64_t M, int64_t N, int64_t K, int nz, hipStream_t s);
hipError_t launch_reduce(const float* part, int nz, int64_t len, float alpha, float* out, hipStream_t s);
hipError_t launch_colsum(const float* X, int64_t M, float* part, int nb, hipStream_t s);
hipError_t launch_train_e1(int64_t M, const float* HD, const float* b1, uint16_t* AD, float* S1, float* T1,
                           hipStream_t s);
hipError_t launch_train_e2(int64_t M, const float* HD, const float* b2, const float* w3, uint16_t* D2, float* HB2,
                           float* DA2, hipStream_t s);
hipError_t launch_train_e3(int64_t M, const float* AB, const float* S1, const float* T1, uint16_t* D1, float* HB1,
                           hipStream_t s);
hipError_t launch_loss(const float* F, const float* Ft, int64_t len, float* delta, float* part, int nb, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, hipStream_t s);
hipError_t launch_refresh(const float* p, uint16_t* W1, uint16_t* W1T, uint16_t* W2, uint16_t* W2T, hipStream_t s);
hipError_t nn_setup();

// a piece of the caller's device memory
struct Span {
    void* p = nullptr;
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// Carves 256-byte aligned pieces off a caller-owned device buffer; with a
// null base it only adds up their sizes (the size queries).
struct SpanCarver {
    char* base;
    size_t off = 0;
    explicit SpanCarver(void* b) : base(static_cast<char*>(b)) {}
    Span take(size_t bytes)
    {
        off = (off + 255) / 256 * 256;
        Span sp;
        sp.p = base ? base + off : nullptr;
        off += bytes;
        return sp;
    }
};

// per-run buffers of the RESPA inner force (caller-owned, pamd_set_mts)
struct MtsBuffers {
    Span G, gG, e, fnn;
};

// r-RESPA buffers of one run of R_cap replicas (n atoms, slab width npad)
inline MtsBuffers carve_mts(SpanCarver& cv, int64_t R_cap, int n, int npad)
{
    const size_t rows = (size_t)R_cap * n;
    MtsBuffers b;
    b.G = cv.take(rows * kFeat * 2);
    b.gG = cv.take(rows * kFeat * 2);
    b.e = cv.take(rows * 4);
    b.fnn = cv.take((size_t)R_cap * 3 * npad * 4);
    return b;
}

}  // namespace nn
}  // namespace pamd

// the surrogate object behind the opaque pamd_nn handle; every device array
// is a piece of the memory the caller passed to pamd_nn_create
struct pamd_nn {
    pamd::nn::Topo topo{};
    pamd::nn::Weights w{};
    float* params = nullptr;   // device FP32 masters [kParams]
    float* grad = nullptr;     // device [kParams]
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    uint16_t* wbf = nullptr;   // device BF16 copies: W1T | W1 | W2T | W2
    int64_t adam_t = 0;
    int64_t max_conf = 0;      // largest batch of the inference / training calls
    // inference / training workspace, sized for max_conf configurations
    pamd::nn::Span GV, gG, e, F, delta, HD, AD, S1, T1, D2, HB2, DA2, D1, HB1, part, colpart, losspart;
    std::string err;
};
