// Host side of the learned multiple-time-step surrogate: the pamd_nn_* calls
// of include/pamd.h (weights, inference, force-matching training).  Every
// device array lives in the memory the caller hands to pamd_nn_create; this
// file allocates no device memory.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "nn_internal.h"
#include "pamd.h"

using namespace pamd::nn;

namespace {

pamd_status nfail(pamd_nn* nn, pamd_status st, const std::string& m)
{
    if (nn)
        nn->err = m;
    return st;
}

#define NNCHK(nn, call)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return nfail(nn, PAMD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

constexpr int kSplitK = 32;     // K slices of the weight-gradient products
constexpr int kColBlocks = 64;  // row blocks of the column sums
constexpr int kLossBlocks = 64;

// array-mode configuration access: [n_conf][n][3]
ConfIO array_io(const float* x, float* f, int64_t count, int n)
{
    ConfIO io{};
    io.xbase[0] = io.xbase[1] = x;
    io.fout = f;
    io.ctl = nullptr;
    io.count = count;
    io.xs_conf = io.fs_conf = 3 * (int64_t)n;
    io.xs_comp = io.fs_comp = 1;
    io.xs_atom = io.fs_atom = 3;
    return io;
}

// Device memory of one surrogate in carve order: FP32 masters, gradient and
// Adam moments (4 x kParams), the BF16 weight copies, then the workspace of
// max_conf configurations (M = max_conf n rows: features and their
// directional derivatives, adjoints, hidden activations of the training
// products, split-K partial sums).  nn == nullptr only counts the bytes.
void carve_nn(SpanCarver& cv, pamd_nn* nn, int n, int64_t max_conf)
{
    const size_t M = (size_t)max_conf * n, len = 3 * M;
    pamd_nn tmp;
    pamd_nn* t = nn ? nn : &tmp;
    const Span params = cv.take(sizeof(float) * 4 * kParams);
    const Span wbf = cv.take(sizeof(uint16_t) * 2 * (kFeat * kH + kH * kH));
    t->GV = cv.take(2 * M * kFeat * 2);
    t->gG = cv.take(M * kFeat * 2);
    t->e = cv.take(M * 4);
    t->F = cv.take(len * 4);
    t->delta = cv.take(len * 4);
    t->HD = cv.take(2 * M * kH * 4);
    t->AD = cv.take(2 * M * kH * 2);
    t->S1 = cv.take(M * kH * 4);
    t->T1 = cv.take(M * kH * 4);
    t->D2 = cv.take(2 * M * kH * 2);
    t->HB2 = cv.take(M * kH * 4);
    t->DA2 = cv.take(M * kH * 4);
    t->D1 = cv.take(2 * M * kH * 2);
    t->HB1 = cv.take(M * kH * 4);
    t->part = cv.take((size_t)kSplitK * kFeat * kH * 4);
    t->colpart = cv.take((size_t)kColBlocks * kH * 4);
    t->losspart = cv.take((size_t)(kLossBlocks + 1) * 4);
    if (nn) {
        nn->params = params.as<float>();
        nn->wbf = wbf.as<uint16_t>();
    }
}

pamd_status check_batch(pamd_nn* nn, int64_t n_conf)
{
    if (n_conf > nn->max_conf)
        return nfail(nn, PAMD_ERR_ARG, "batch of " + std::to_string(n_conf) + " configurations exceeds max_conf = " +
                                           std::to_string(nn->max_conf) + " given to pamd_nn_create");
    return PAMD_OK;
}

// energies and forces of n_conf configurations into F (array layout); the
// feature rows go to G, dE/dG to gG, row energies to e (M = n_conf n rows each)
pamd_status infer_into(pamd_nn* nn, int64_t n_conf, const float* d_x, float* d_F, float* d_E, uint16_t* G,
                       uint16_t* gG, float* e, hipStream_t s)
{
    const int n = nn->topo.n;
    const int64_t M = n_conf * n;
    const ConfIO io = array_io(d_x, d_F, n_conf, n);
    NNCHK(nn, launch_features(nn->topo, io, n_conf, nullptr, G, s));
    NNCHK(nn, launch_mlp(nn->w, G, gG, e, nullptr, M, n, s));
    NNCHK(nn, launch_force(nn->topo, io, n_conf, gG, e, d_E, s));
    return PAMD_OK;
}

pamd_status infer(pamd_nn* nn, int64_t n_conf, const float* d_x, float* d_F, float* d_E, hipStream_t s)
{
    return infer_into(nn, n_conf, d_x, d_F, d_E, nn->GV.as<uint16_t>(), nn->gG.as<uint16_t>(), nn->e.as<float>(), s);
}

// ---- allocation-free inference (pamd_nn_forces_static) -------------------
// Its staging rows live in one file-scope device array, a copy per GPU held
// until the process ends.  In host code the array's name is no device
// address: each device's copy is looked up once with hipGetSymbolAddress
// (with that device current) and only that pointer is handed to kernels.
constexpr size_t kStaticBytes = (size_t)16 << 20;
static_assert((size_t)PAMD_NN_STATIC_ROWS * (2 * kFeat * 2 + 4) + 3 * 256 <= kStaticBytes,
              "static staging rows exceed the fixed array");
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// this device's copy of `scratch` (looked up on the first call per device)
hipError_t static_scratch(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

pamd_status pamd_nn_query_sizes(int32_t n_atoms, int64_t max_conf, size_t* bytes)
{
    if (!bytes || n_atoms < 1 || n_atoms > kMaxN || max_conf < 1)
        return PAMD_ERR_ARG;
    SpanCarver cv(nullptr);
    carve_nn(cv, nullptr, n_atoms, max_conf);
    *bytes = cv.off;
    return PAMD_OK;
}

pamd_status pamd_nn_create(const pamd_system* sys, const int32_t* atom_type, int64_t max_conf, void* d_mem,
                           size_t mem_bytes, void* stream, pamd_nn** out)
{
    if (!sys || !atom_type || !out)
        return PAMD_ERR_ARG;
    *out = nullptr;
    const int n = sys->n_atoms;
    if (n < 1 || n > kMaxN || (sys->n_bonds > 0 && !sys->bond_idx) || max_conf < 1 || !d_mem ||
        (reinterpret_cast<uintptr_t>(d_mem) & 255) != 0)
        return PAMD_ERR_ARG;
    size_t need = 0;
    if (pamd_nn_query_sizes(n, max_conf, &need) != PAMD_OK || mem_bytes < need)
        return PAMD_ERR_ARG;
    for (int a = 0; a < n; ++a)
        if (atom_type[a] < 0 || atom_type[a] >= kTypes)
            return PAMD_ERR_ARG;
    for (int b = 0; b < 2 * sys->n_bonds; ++b)
        if (sys->bond_idx[b] < 0 || sys->bond_idx[b] >= n)
            return PAMD_ERR_ARG;
    pamd_nn* nn = new pamd_nn();
    Topo& tp = nn->topo;
    tp.n = n;
    // atoms in type order, with the start of each type
    std::vector<int> order(n);
    for (int a = 0; a < n; ++a)
        order[a] = a;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return atom_type[a] < atom_type[b]; });
    for (int a = 0; a < n; ++a) {
        tp.order[a] = (uint8_t)order[a];
        tp.atype[a] = (uint8_t)atom_type[a];
    }
    for (int t = 0; t <= kTypes; ++t)
        tp.tstart[t] = (int32_t)std::count_if(atom_type, atom_type + n, [&](int32_t v) { return v < t; });
    // pairs without a feature: graph distance <= 2 through the bonds (self, 1-2, 1-3)
    std::vector<std::vector<int>> adj(n);
    for (int b = 0; b < sys->n_bonds; ++b) {
        adj[sys->bond_idx[2 * b]].push_back(sys->bond_idx[2 * b + 1]);
        adj[sys->bond_idx[2 * b + 1]].push_back(sys->bond_idx[2 * b]);
    }
    std::vector<std::vector<char>> excl(n, std::vector<char>(n, 0));
    for (int i = 0; i < n; ++i) {
        std::vector<int> dist(n, -1);
        std::vector<int> q{i};
        dist[i] = 0;
        for (size_t h = 0; h < q.size(); ++h)
            for (int j : adj[q[h]])
                if (dist[j] < 0) {
                    dist[j] = dist[q[h]] + 1;
                    q.push_back(j);
                }
        for (int j = 0; j < n; ++j)
            if (dist[j] >= 0 && dist[j] <= 2)
                excl[i][j] = 1;
    }
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            if (excl[order[p]][order[q]])
                tp.excl[p][q >> 5] |= 1u << (q & 31);
    // parameters (zero) and BF16 copies in the caller's memory
    SpanCarver cv(d_mem);
    carve_nn(cv, nn, n, max_conf);
    nn->max_conf = max_conf;
    hipStream_t s = as_stream(stream);
    hipError_t e = hipMemsetAsync(nn->params, 0, sizeof(float) * 4 * kParams, s);
    if (e == hipSuccess)
        e = hipMemsetAsync(nn->wbf, 0, sizeof(uint16_t) * 2 * (kFeat * kH + kH * kH), s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = nn_setup();
    void* sp = nullptr;   // this device's allocation-free staging array (set up once per device)
    if (e == hipSuccess)
        e = static_scratch(&sp);
    if (e != hipSuccess) {
        delete nn;
        return PAMD_ERR_HIP;
    }
    nn->grad = nn->params + kParams;
    nn->adam_m = nn->params + 2 * kParams;
    nn->adam_v = nn->params + 3 * kParams;
    uint16_t* b = nn->wbf;
    nn->w.W1T = b;
    nn->w.W1 = b + kFeat * kH;
    nn->w.W2T = b + 2 * kFeat * kH;
    nn->w.W2 = b + 2 * kFeat * kH + kH * kH;
    nn->w.b1 = nn->params + ob1;
    nn->w.b2 = nn->params + ob2;
    nn->w.w3 = nn->params + ow3;
    nn->w.b3 = nn->params + ob3;
    *out = nn;
    return PAMD_OK;
}

pamd_status pamd_nn_set_weights(pamd_nn* nn, const float* params, void* stream)
{
    if (!nn || !params)
        return nfail(nn, PAMD_ERR_ARG, "null argument");
    hipStream_t s = as_stream(stream);
    NNCHK(nn, hipMemcpyAsync(nn->params, params, sizeof(float) * kParams, hipMemcpyHostToDevice, s));
    NNCHK(nn, hipMemsetAsync(nn->adam_m, 0, sizeof(float) * 2 * kParams, s));
    nn->adam_t = 0;
    uint16_t* b = nn->wbf;
    NNCHK(nn, launch_refresh(nn->params, b + kFeat * kH, b, b + 2 * kFeat * kH + kH * kH, b + 2 * kFeat * kH, s));
    NNCHK(nn, hipStreamSynchronize(s));
    return PAMD_OK;
}

pamd_status pamd_nn_get_weights(pamd_nn* nn, float* params, void* stream)
{
    if (!nn || !params)
        return nfail(nn, PAMD_ERR_ARG, "null argument");
    hipStream_t s = as_stream(stream);
    NNCHK(nn, hipMemcpyAsync(params, nn->params, sizeof(float) * kParams, hipMemcpyDeviceToHost, s));
    NNCHK(nn, hipStreamSynchronize(s));
    return PAMD_OK;
}

pamd_status pamd_nn_forces(pamd_nn* nn, int64_t n_conf, const float* d_x, float* d_F, float* d_E, void* stream)
{
    if (!nn)
        return PAMD_ERR_ARG;
    if (n_conf < 0 || (n_conf > 0 && (!d_x || !d_F)))
        return nfail(nn, PAMD_ERR_ARG, "bad configuration arrays");
    if (n_conf == 0)
        return PAMD_OK;
    if (check_batch(nn, n_conf) != PAMD_OK)
        return PAMD_ERR_ARG;
    return infer(nn, n_conf, d_x, d_F, d_E, as_stream(stream));
}

pamd_status pamd_nn_forces_static(pamd_nn* nn, int64_t n_conf, const float* d_x, float* d_F, float* d_E,
                                  void* stream)
{
    if (!nn)
        return PAMD_ERR_ARG;
    if (n_conf < 0 || (n_conf > 0 && (!d_x || !d_F)))
        return nfail(nn, PAMD_ERR_ARG, "bad configuration arrays");
    const int64_t rows = n_conf * nn->topo.n;
    if (rows > PAMD_NN_STATIC_ROWS)
        return nfail(nn, PAMD_ERR_ARG, "n_conf * n_atoms = " + std::to_string(rows) +
                                           " exceeds the fixed staging of PAMD_NN_STATIC_ROWS = " +
                                           std::to_string(PAMD_NN_STATIC_ROWS) + " rows");
    if (n_conf == 0)
        return PAMD_OK;
    void* base = nullptr;
    NNCHK(nn, static_scratch(&base));
    // every staged value is written by the features / MLP kernels of this
    // call before it is read, so nothing needs clearing between calls
    SpanCarver cv(base);
    const Span G = cv.take((size_t)rows * kFeat * 2);
    const Span gG = cv.take((size_t)rows * kFeat * 2);
    const Span e = cv.take((size_t)rows * 4);
    return infer_into(nn, n_conf, d_x, d_F, d_E, G.as<uint16_t>(), gG.as<uint16_t>(), e.as<float>(),
                      as_stream(stream));
}

pamd_status pamd_nn_loss_grad(pamd_nn* nn, int64_t n_conf, const float* d_x, const float* d_F_target,
                              float* d_loss, float* d_grad, void* stream)
{
    if (!nn)
        return PAMD_ERR_ARG;
    if (n_conf < 1 || !d_x || !d_F_target || !d_loss)
        return nfail(nn, PAMD_ERR_ARG, "bad arguments");
    if (check_batch(nn, n_conf) != PAMD_OK)
        return PAMD_ERR_ARG;
    hipStream_t s = as_stream(stream);
    const int n = nn->topo.n;
    const int64_t M = n_conf * n;
    const int64_t len = M * 3;
    pamd_status st = infer(nn, n_conf, d_x, nn->F.as<float>(), nullptr, s);
    if (st != PAMD_OK)
        return st;
    NNCHK(nn, launch_loss(nn->F.as<float>(), d_F_target, len, nn->delta.as<float>(), nn->losspart.as<float>(),
                          kLossBlocks, s));
    NNCHK(nn, launch_reduce(nn->losspart.as<float>(), kLossBlocks, 1, 1.0f, d_loss, s));
    if (!d_grad)
        return PAMD_OK;

    // directional derivative of the features along delta = dL/dF: rows M..2M-1 of GV
    uint16_t* GV = nn->GV.as<uint16_t>();
    const ConfIO io = array_io(d_x, nullptr, n_conf, n);
    NNCHK(nn, launch_features(nn->topo, io, n_conf, nn->delta.as<float>(), GV + (size_t)M * kFeat, s));
    float* HD = nn->HD.as<float>();
    uint16_t* AD = nn->AD.as<uint16_t>();
    uint16_t* D2 = nn->D2.as<uint16_t>();
    uint16_t* D1 = nn->D1.as<uint16_t>();
    float* part = nn->part.as<float>();
    float* colpart = nn->colpart.as<float>();
    const Weights& w = nn->w;
    // forward and its derivative: [h1 ; dh1] = [G ; v] W1
    NNCHK(nn, launch_gemm(GV, kFeat, 1, w.W1, kH, 1, HD, 2 * M, kH, kFeat, 1, s));
    NNCHK(nn, launch_train_e1(M, HD, w.b1, AD, nn->S1.as<float>(), nn->T1.as<float>(), s));
    // [h2 ; dh2] = [a1 ; da1] W2
    NNCHK(nn, launch_gemm(AD, kH, 1, w.W2, kH, 1, HD, 2 * M, kH, kH, 1, s));
    NNCHK(nn, launch_train_e2(M, HD, w.b2, w.w3, D2, nn->HB2.as<float>(), nn->DA2.as<float>(), s));
    // adjoints into layer 1: [abar1 ; dadot1] = [hbar2 ; dhdot2] W2^T
    NNCHK(nn, launch_gemm(D2, kH, 1, w.W2T, kH, 1, HD, 2 * M, kH, kH, 1, s));
    NNCHK(nn, launch_train_e3(M, HD, nn->S1.as<float>(), nn->T1.as<float>(), D1, nn->HB1.as<float>(), s));
    // dL/dW = -(d/dW of the directional derivative of E along v)
    NNCHK(nn, launch_gemm(GV, 1, kFeat, D1, kH, 1, part, kFeat, kH, 2 * M, kSplitK, s));
    NNCHK(nn, launch_reduce(part, kSplitK, (int64_t)kFeat * kH, -1.0f, d_grad + oW1, s));
    NNCHK(nn, launch_gemm(AD, 1, kH, D2, kH, 1, part, kH, kH, 2 * M, kSplitK, s));
    NNCHK(nn, launch_reduce(part, kSplitK, (int64_t)kH * kH, -1.0f, d_grad + oW2, s));
    NNCHK(nn, launch_colsum(nn->HB1.as<float>(), M, colpart, kColBlocks, s));
    NNCHK(nn, launch_reduce(colpart, kColBlocks, kH, -1.0f, d_grad + ob1, s));
    NNCHK(nn, launch_colsum(nn->HB2.as<float>(), M, colpart, kColBlocks, s));
    NNCHK(nn, launch_reduce(colpart, kColBlocks, kH, -1.0f, d_grad + ob2, s));
    NNCHK(nn, launch_colsum(nn->DA2.as<float>(), M, colpart, kColBlocks, s));
    NNCHK(nn, launch_reduce(colpart, kColBlocks, kH, -1.0f, d_grad + ow3, s));
    // b3 moves every energy alike: no force depends on it
    NNCHK(nn, launch_reduce(colpart, 0, 1, 0.0f, d_grad + ob3, s));
    return PAMD_OK;
}

pamd_status pamd_nn_train_step(pamd_nn* nn, int64_t n_conf, const float* d_x, const float* d_F_target, float lr,
                               float* d_loss, void* stream)
{
    if (!nn)
        return PAMD_ERR_ARG;
    if (!(lr > 0.0f))
        return nfail(nn, PAMD_ERR_ARG, "lr must be > 0");
    hipStream_t s = as_stream(stream);
    float* loss = d_loss ? d_loss : nn->losspart.as<float>() + kLossBlocks;
    pamd_status st = pamd_nn_loss_grad(nn, n_conf, d_x, d_F_target, loss, nn->grad, stream);
    if (st != PAMD_OK)
        return st;
    nn->adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float bc1 = (float)(1.0 - pow(b1, (double)nn->adam_t));
    const float bc2 = (float)(1.0 - pow(b2, (double)nn->adam_t));
    NNCHK(nn, launch_adam(nn->params, nn->grad, nn->adam_m, nn->adam_v, kParams, lr, (float)b1, (float)b2, 1e-8f,
                          bc1, bc2, s));
    uint16_t* b = nn->wbf;
    NNCHK(nn, launch_refresh(nn->params, b + kFeat * kH, b, b + 2 * kFeat * kH + kH * kH, b + 2 * kFeat * kH, s));
    return PAMD_OK;
}

// The caller's memory stays the caller's: only the host object is freed.
void pamd_nn_destroy(pamd_nn* nn)
{
    delete nn;
}

const char* pamd_nn_last_error(const pamd_nn* nn) { return nn ? nn->err.c_str() : "null surrogate"; }

}  // extern "C"
