// Host side of the learned multiple-time-step surrogate: the pamd_nn_* calls
// of include/pamd.h (weights, inference, force-matching training).
#include <math.h>
#include <string.h>

#include <algorithm>
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

// energies and forces of n_conf configurations into F (array layout); G rows
// go to the first half of nn->GV
pamd_status infer(pamd_nn* nn, int64_t n_conf, const float* d_x, float* d_F, float* d_E, hipStream_t s)
{
    const int n = nn->topo.n;
    const int64_t M = n_conf * n;
    NNCHK(nn, nn->GV.need((size_t)2 * M * kFeat * 2, s));
    NNCHK(nn, nn->gG.need((size_t)M * kFeat * 2, s));
    NNCHK(nn, nn->e.need((size_t)M * 4, s));
    const ConfIO io = array_io(d_x, d_F, n_conf, n);
    NNCHK(nn, launch_features(nn->topo, io, n_conf, nullptr, nn->GV.as<uint16_t>(), s));
    NNCHK(nn, launch_mlp(nn->w, nn->GV.as<uint16_t>(), nn->gG.as<uint16_t>(), nn->e.as<float>(), nullptr, M, n, s));
    NNCHK(nn, launch_force(nn->topo, io, n_conf, nn->gG.as<uint16_t>(), nn->e.as<float>(), d_E, s));
    return PAMD_OK;
}

}  // namespace

extern "C" {

pamd_status pamd_nn_create(const pamd_system* sys, const int32_t* atom_type, pamd_nn** out)
{
    if (!sys || !atom_type || !out)
        return PAMD_ERR_ARG;
    *out = nullptr;
    const int n = sys->n_atoms;
    if (n < 1 || n > kMaxN || (sys->n_bonds > 0 && !sys->bond_idx))
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
    // device parameters (zero) and BF16 copies
    hipError_t e = hipMalloc(&nn->params, sizeof(float) * 4 * kParams);
    if (e == hipSuccess)
        e = hipMalloc(&nn->wbf, sizeof(uint16_t) * 2 * (kFeat * kH + kH * kH));
    if (e == hipSuccess)
        e = hipMemset(nn->params, 0, sizeof(float) * 4 * kParams);
    if (e == hipSuccess)
        e = hipMemset(nn->wbf, 0, sizeof(uint16_t) * 2 * (kFeat * kH + kH * kH));
    if (e == hipSuccess)
        e = nn_setup();
    if (e != hipSuccess) {
        pamd_nn_destroy(nn);
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
    return infer(nn, n_conf, d_x, d_F, d_E, as_stream(stream));
}

pamd_status pamd_nn_loss_grad(pamd_nn* nn, int64_t n_conf, const float* d_x, const float* d_F_target,
                              float* d_loss, float* d_grad, void* stream)
{
    if (!nn)
        return PAMD_ERR_ARG;
    if (n_conf < 1 || !d_x || !d_F_target || !d_loss)
        return nfail(nn, PAMD_ERR_ARG, "bad arguments");
    hipStream_t s = as_stream(stream);
    const int n = nn->topo.n;
    const int64_t M = n_conf * n;
    const int64_t len = M * 3;
    NNCHK(nn, nn->F.need((size_t)len * 4, s));
    NNCHK(nn, nn->delta.need((size_t)len * 4, s));
    NNCHK(nn, nn->losspart.need((size_t)kLossBlocks * 4, s));
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
    NNCHK(nn, nn->HD.need((size_t)2 * M * kH * 4, s));
    NNCHK(nn, nn->AD.need((size_t)2 * M * kH * 2, s));
    NNCHK(nn, nn->S1.need((size_t)M * kH * 4, s));
    NNCHK(nn, nn->T1.need((size_t)M * kH * 4, s));
    NNCHK(nn, nn->D2.need((size_t)2 * M * kH * 2, s));
    NNCHK(nn, nn->HB2.need((size_t)M * kH * 4, s));
    NNCHK(nn, nn->DA2.need((size_t)M * kH * 4, s));
    NNCHK(nn, nn->D1.need((size_t)2 * M * kH * 2, s));
    NNCHK(nn, nn->HB1.need((size_t)M * kH * 4, s));
    NNCHK(nn, nn->part.need((size_t)kSplitK * kFeat * kH * 4, s));
    NNCHK(nn, nn->colpart.need((size_t)kColBlocks * kH * 4, s));
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
    NNCHK(nn, nn->losspart.need((size_t)(kLossBlocks + 1) * 4, s));
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

void pamd_nn_destroy(pamd_nn* nn)
{
    if (!nn)
        return;
    (void)hipDeviceSynchronize();
    if (nn->params)
        (void)hipFree(nn->params);
    if (nn->wbf)
        (void)hipFree(nn->wbf);
    for (DevBuf* b : {&nn->GV, &nn->gG, &nn->e, &nn->F, &nn->delta, &nn->HD, &nn->AD, &nn->S1, &nn->T1, &nn->D2,
                      &nn->HB2, &nn->DA2, &nn->D1, &nn->HB1, &nn->part, &nn->colpart, &nn->losspart})
        b->release();
    delete nn;
}

const char* pamd_nn_last_error(const pamd_nn* nn) { return nn ? nn->err.c_str() : "null surrogate"; }

}  // extern "C"
