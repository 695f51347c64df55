// Host runtime of libpamd: the C ABI declared in include/pamd.h.
//
// Owns no device memory: the caller's d_state / d_work buffers are carved
// into per-run regions (256-byte aligned).  Builds, per run, the exclusion
// and 1-4 lists from the bond graph, the per-tile pair-coefficient table of
// the MD kernel and the bonded-term records, then drives the kernels of
// md_kernel.hip (PAMD step 3) and resample.hip (steps 1, 2, 4).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "nn_internal.h"
#include "pamd.h"
#include "pamd_internal.h"

namespace {
// Named range of one C-ABI call in the ROCm marker trace (rocprofv3
// --marker-trace): host-side enqueue of the call's kernels; without a tracing
// tool attached the push and pop do nothing.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};
}  // namespace

namespace pamd {
hipError_t launch_md(const RunDev<float>& d, int n_steps, int blocks, int waves, hipStream_t s);
hipError_t launch_md(const RunDev<double>& d, int n_steps, int blocks, int waves, hipStream_t s);
hipError_t launch_energy(const RunDev<float>& d, int blocks, int waves, hipStream_t s);
hipError_t launch_energy(const RunDev<double>& d, int blocks, int waves, hipStream_t s);
hipError_t launch_forces(const RunDev<float>& d, int64_t r0, int count, int waves, hipStream_t s);
hipError_t launch_forces(const RunDev<double>& d, int64_t r0, int count, int waves, hipStream_t s);
hipError_t md_occupancy(int precision_fp32, int nslot, int diel, int n, int waves, int* blocks_per_cu);
size_t md_lds(int precision_fp32, int nslot, int n, int waves);
hipError_t launch_init(const RunDev<float>& d, hipStream_t s);
hipError_t launch_init(const RunDev<double>& d, hipStream_t s);
hipError_t launch_resample(const RunDev<float>& d, double T_req, double mtot, hipStream_t s);
hipError_t launch_resample(const RunDev<double>& d, double T_req, double mtot, hipStream_t s);
size_t part_doubles(int64_t R_cap);
size_t cpart_count(int64_t R_cap);
hipError_t launch_md_begin(const RunDev<float>& d, hipStream_t s);
hipError_t launch_md_begin(const RunDev<double>& d, hipStream_t s);
hipError_t launch_md_finalize(const RunDev<float>& d, int n, hipStream_t s);
hipError_t launch_md_finalize(const RunDev<double>& d, int n, hipStream_t s);
hipError_t launch_observables(const RunDev<float>& d, hipStream_t s);
hipError_t launch_observables(const RunDev<double>& d, hipStream_t s);
hipError_t launch_respa(const RunDev<float>& d, const float* fnn, int ops, uint32_t step_off, double dt_outer,
                        uint32_t p24_outer, int blocks, int waves, hipStream_t s);
hipError_t launch_export(const RunDev<float>& d, int64_t r0, int64_t count, float* xo, float* fo, int waves,
                         hipStream_t s);
size_t wide_lds_bytes(int nmax, int waves, int ljsz);
hipError_t wide_setup(int diel, int nmax, int waves, int ljsz, int* blocks_per_cu);
hipError_t launch_md_wide(const RunDev<float>* runs, const int32_t* order, int n_runs, int32_t* counter, int nmax,
                          int n_steps, int diel, int lang, int ljsz, int blocks, int waves, hipStream_t s);
hipError_t launch_forces_wide(const RunDev<float>& d, int64_t r0, int count, int nmax, int waves, int ljsz,
                              hipStream_t s);
}  // namespace pamd

using namespace pamd;

namespace {

constexpr size_t kAlign = 256;

struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <typename T>
    T* take(size_t count)
    {
        off = (off + kAlign - 1) / kAlign * kAlign;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// host copies of the per-run tables (FP64; cast to the kernel precision on upload)
struct HostTables {
    int n = 0, npad = 0, nslot = 0;
    int wide = 0, nchunk = 0;
    std::vector<double> atomp;           // wide layout: [n][2] per-atom Coulomb factor and LJ class
    std::vector<double> lj;              // wide layout: [rows][lj_stride_of(rows)][2] LJ class table
    std::vector<uint32_t> pmask;         // wide layout: [n][nchunk][2] exclusion / 1-4 bits
    std::vector<uint64_t> stepmask;      // wide layout: [t][s] rotation steps that need the masks
    std::vector<double> ab, c;           // [steps][16][2], [steps][16]
    std::vector<int32_t> bidx, aidx, didx;  // int4 records (dihedrals: two per group slot)
    std::vector<double> bpar, apar, dpar;   // dihedrals: 45 per group slot
    int n6 = 0;                          // angle slots of the six-angle body
    std::vector<double> mass, x_init;
    double mtot = 0;
};

struct Run {
    RunDev<float> f{};
    RunDev<double> d{};
    HostTables tab;
    double mtot = 0;
    double nu = 0;                   // Andersen collision frequency
    pamd::nn::MtsBuffers mts;        // r-RESPA buffers (surrogate attached)
};

}  // namespace

constexpr int kGraphSlots = 4;

struct pamd_ctx {
    hipGraph_t graph[kGraphSlots] = {};
    hipGraphExec_t graph_exec[kGraphSlots] = {};
    int n_runs = 0;
    int fp32 = 1;
    std::vector<Run> runs;
    std::string err;
    int failed = 0;
    int n_cu = 0;
    int have_energy = 0;     // some pamd_md_steps (or a state with energies) since init
    pamd_nn* nn = nullptr;   // learned surrogate of the r-RESPA inner force (null: plain MD)
    int mts_ratio = 0;       // inner steps per outer step
    // launch shapes: register-tile runs (k_md, one launch per run) and wide
    // runs (every one of them in one persistent k_md_wide launch)
    int tile_waves = 0, tile_blocks = 0;
    size_t tile_lds = 0;
    int wide_waves = 0, wide_blocks = 0;
    size_t wide_lds = 0;
    int wide = 0, n_wide = 0, nmax = 0, diel = 0;   // wide: some run is wide; nmax: largest wide molecule
    int lj_rows = 0;                   // LJ class-table rows of the wide runs (largest class count + 1)
    RunDev<float>* d_runs = nullptr;   // device copies of the runs' descriptors
    int32_t* d_order = nullptr;        // runs in decreasing pair work
    int32_t* d_counter = nullptr;      // work-queue counter
    // the register-tile runs of a context with several of them run on side
    // streams forked from and joined back to the caller's stream, so their
    // persistent launches (each latency-bound on a fraction of the CUs for a
    // small population) overlap; the wide launch goes on the caller's stream
    // after the fork and before the join: its workgroups take the CUs the
    // tile launches leave free and, through its work queue, the rest as those
    // finish
    static constexpr int kSide = 3;
    int n_side = 0;
    hipStream_t side[kSide] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kSide] = {};
};

namespace {

pamd_status fail(pamd_ctx* c, pamd_status st, const std::string& msg)
{
    if (c) {
        c->err = msg;
        if (st != PAMD_ERR_ARG)
            c->failed = st;
    }
    return st;
}

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ctx, PAMD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

int nslot_of(int n) { return (n + kRow - 1) / kRow; }
int npad_of(int n, int wide) { return wide ? (n + kWide - 1) / kWide * kWide : nslot_of(n) * kRow; }

// MD layout of run r: PAMD_LAYOUT_WIDE / TILE as asked; AUTO takes the wide
// layout when the context holds a molecule above the register-tile limit
int run_is_wide(const pamd_system* sys, const pamd_params* p, int n_runs, int r)
{
    if (p[0].precision != PAMD_FP32)
        return 0;
    if (sys[r].n_atoms > PAMD_TILE_ATOMS || p[r].layout == PAMD_LAYOUT_WIDE)
        return 1;
    if (p[r].layout == PAMD_LAYOUT_TILE)
        return 0;
    for (int q = 0; q < n_runs; ++q)
        if (sys[q].n_atoms > PAMD_TILE_ATOMS)
            return 1;
    return 0;
}

// LJ classes: the distinct per-atom (sigma, epsilon) values in order of first
// appearance; cls[a] = class of atom a.  Returns the number of classes.
int lj_classes(const pamd_system& s, std::vector<int>* cls)
{
    std::vector<std::pair<double, double>> seen;
    if (cls)
        cls->assign(s.n_atoms, 0);
    for (int a = 0; a < s.n_atoms; ++a) {
        const std::pair<double, double> v(s.sigma[a], s.epsilon[a]);
        int k = 0;
        while (k < (int)seen.size() && seen[k] != v)
            ++k;
        if (k == (int)seen.size())
            seen.push_back(v);
        if (cls)
            (*cls)[a] = k;
    }
    return (int)seen.size();
}

// graph distance (capped at 4) between every pair of atoms of the bond graph
std::vector<int> graph_distance(int n, int nb, const int32_t* bidx)
{
    std::vector<std::vector<int>> adj(n);
    for (int t = 0; t < nb; ++t) {
        adj[bidx[2 * t]].push_back(bidx[2 * t + 1]);
        adj[bidx[2 * t + 1]].push_back(bidx[2 * t]);
    }
    std::vector<int> dist((size_t)n * n, 4);
    for (int s = 0; s < n; ++s) {
        dist[(size_t)s * n + s] = 0;
        std::vector<int> front{s};
        for (int depth = 1; depth <= 3; ++depth) {
            std::vector<int> next;
            for (int u : front)
                for (int w : adj[u])
                    if (dist[(size_t)s * n + w] > depth) {
                        dist[(size_t)s * n + w] = depth;
                        next.push_back(w);
                    }
            front.swap(next);
        }
    }
    return dist;
}

pamd_status validate(pamd_ctx* c, const pamd_system& s, const pamd_params& p, int fp32)
{
    if (s.n_atoms < 1 || s.n_atoms > PAMD_MAX_ATOMS)
        return fail(c, PAMD_ERR_ARG, "n_atoms must be in 1.." + std::to_string(PAMD_MAX_ATOMS));
    if (!fp32 && s.n_atoms > PAMD_TILE_ATOMS)
        return fail(c, PAMD_ERR_ARG, "molecules above " + std::to_string(PAMD_TILE_ATOMS) + " atoms need FP32");
    if (!fp32 && s.n_atoms > 2 * kRow)
        return fail(c, PAMD_ERR_ARG, "FP64 precision supports at most 32 atoms");
    if (!s.mass || !s.charge || !s.sigma || !s.epsilon || !s.x_init)
        return fail(c, PAMD_ERR_ARG, "null per-atom array");
    if (s.n_bonds < 0 || s.n_angles < 0 || s.n_dihedrals < 0)
        return fail(c, PAMD_ERR_ARG, "negative term count");
    if ((s.n_bonds && (!s.bond_idx || !s.bond_k || !s.bond_r0)) ||
        (s.n_angles && (!s.angle_idx || !s.angle_k || !s.angle_theta0)) ||
        (s.n_dihedrals && (!s.dih_idx || !s.dih_k || !s.dih_n || !s.dih_delta)))
        return fail(c, PAMD_ERR_ARG, "null term array");
    for (int a = 0; a < s.n_atoms; ++a)
        if (!(s.mass[a] > 0.0) || !(s.epsilon[a] >= 0.0))
            return fail(c, PAMD_ERR_ARG, "mass must be > 0 and epsilon >= 0");
    auto in_range = [&](const int32_t* idx, int count, int k) {
        for (int i = 0; i < count * k; ++i)
            if (idx[i] < 0 || idx[i] >= s.n_atoms)
                return false;
        return true;
    };
    if (!in_range(s.bond_idx, s.n_bonds, 2) || !in_range(s.angle_idx, s.n_angles, 3) ||
        !in_range(s.dih_idx, s.n_dihedrals, 4))
        return fail(c, PAMD_ERR_ARG, "term index out of range");
    for (int t = 0; t < s.n_dihedrals; ++t) {
        if (s.dih_n[t] < 1 || s.dih_n[t] > 6)
            return fail(c, PAMD_ERR_ARG, "dihedral multiplicity must be 1..6");
        if (fabs(sin(s.dih_delta[t])) > 1e-9)
            return fail(c, PAMD_ERR_ARG, "dihedral phase must be 0 or pi");
    }
    if (s.dielectric != PAMD_DIELECTRIC_VACUUM && s.dielectric != PAMD_DIELECTRIC_4R)
        return fail(c, PAMD_ERR_ARG, "unknown dielectric mode");
    if (p.R_target < 1 || p.R_cap < p.R_target || p.R_cap > (int64_t)1 << 30)
        return fail(c, PAMD_ERR_ARG, "need 1 <= R_target <= R_cap <= 2^30");
    if (!(p.T0 > 0) || !(p.dt > 0) || !(p.nu >= 0) || !(s.kB > 0))
        return fail(c, PAMD_ERR_ARG, "T0, dt, kB must be > 0 and nu >= 0");
    if (p.waves_per_block < 0 || p.waves_per_block > 16)
        return fail(c, PAMD_ERR_ARG, "waves_per_block must be 0..16");
    if (p.resampling < PAMD_RESAMPLE_NEAREST || p.resampling > PAMD_RESAMPLE_NONE)
        return fail(c, PAMD_ERR_ARG, "unknown resampling mode");
    if (p.thermostat != PAMD_THERMOSTAT_ANDERSEN && p.thermostat != PAMD_THERMOSTAT_LANGEVIN)
        return fail(c, PAMD_ERR_ARG, "unknown thermostat");
    if (p.layout < PAMD_LAYOUT_AUTO || p.layout > PAMD_LAYOUT_WIDE)
        return fail(c, PAMD_ERR_ARG, "unknown layout");
    if (p.layout == PAMD_LAYOUT_TILE && s.n_atoms > PAMD_TILE_ATOMS)
        return fail(c, PAMD_ERR_ARG, "the register-tile layout takes at most " + std::to_string(PAMD_TILE_ATOMS) +
                                         " atoms");
    if (p.layout == PAMD_LAYOUT_WIDE && !fp32)
        return fail(c, PAMD_ERR_ARG, "the wide layout is FP32 only");
    if (p.wide_waves_per_block < 0 || p.wide_waves_per_block > 4)
        return fail(c, PAMD_ERR_ARG, "wide_waves_per_block must be 0..4");
    return PAMD_OK;
}

// Pack terms of k atoms into passes of W lanes such that no two terms of a
// pass share an atom in the same role (position in the term); a term may be
// stored reversed (a bond, angle or dihedral read backwards is the same
// term).  Empty lanes get index -1.  Returns the packed records
// (4 indices + 2 parameters per slot).
// First fit of bonded terms into passes of W lanes in which no two lanes name
// the same atom in the same role (a term may be reversed).  Returns the passes
// as lists of (term, reversed).
struct Packing {
    std::vector<std::vector<std::pair<int, int>>> passes;
};

static Packing first_fit(int k, const int32_t* idx, const std::vector<int>& order, int W)
{
    constexpr int kWords = (PAMD_MAX_ATOMS + 63) / 64;
    struct Used {
        uint64_t bits[4][kWords];
    };
    Packing pk;
    std::vector<Used> used;
    for (int t : order) {
        const int32_t* a = idx + (size_t)t * k;
        bool placed = false;
        for (int o = 0; o < 2 && !placed; ++o) {
            for (size_t b = 0; b < pk.passes.size() && !placed; ++b) {
                if (pk.passes[b].size() >= (size_t)W)
                    continue;
                bool ok = true;
                for (int r = 0; r < k && ok; ++r) {
                    const int at = o ? a[k - 1 - r] : a[r];
                    ok = !((used[b].bits[r][at >> 6] >> (at & 63)) & 1u);
                }
                if (ok) {
                    for (int r = 0; r < k; ++r) {
                        const int at = o ? a[k - 1 - r] : a[r];
                        used[b].bits[r][at >> 6] |= (uint64_t)1 << (at & 63);
                    }
                    pk.passes[b].push_back({t, o});
                    placed = true;
                }
            }
        }
        if (!placed) {
            Used u;
            memset(&u, 0, sizeof(u));
            for (int r = 0; r < k; ++r)
                u.bits[r][a[r] >> 6] |= (uint64_t)1 << (a[r] & 63);
            used.push_back(u);
            pk.passes.push_back({{t, 0}});
        }
    }
    return pk;
}

// Bonded-term records in passes of W lanes (one term per lane, -1 = empty).
// The number of passes depends on the order in which first fit sees the terms,
// so a fixed set of orders is tried and the one with the fewest passes kept:
// the given order, most-constrained first (terms whose atoms carry the most
// terms), and 62 shuffles from a fixed-seed xorshift generator.  Deterministic.
void pack_terms(int count, int k, const int32_t* idx, const double* p0, const double* p1,
                std::vector<int32_t>& rec, std::vector<double>& par, int W)
{
    Packing best;
    if (count > 0) {
        std::vector<int> order(count);
        for (int t = 0; t < count; ++t)
            order[t] = t;
        best = first_fit(k, idx, order, W);
        std::vector<int> deg(PAMD_MAX_ATOMS, 0);
        for (int t = 0; t < count * k; ++t)
            ++deg[idx[t]];
        std::vector<int> mcf = order;
        std::stable_sort(mcf.begin(), mcf.end(), [&](int a, int b) {
            int da = 0, db = 0;
            for (int r = 0; r < k; ++r) {
                da += deg[idx[(size_t)a * k + r]];
                db += deg[idx[(size_t)b * k + r]];
            }
            return da > db;
        });
        Packing p = first_fit(k, idx, mcf, W);
        if (p.passes.size() < best.passes.size())
            best = p;
        uint64_t st = 0x9E3779B97F4A7C15ull ^ ((uint64_t)count << 8 ^ (uint64_t)k);
        for (int trial = 0; trial < 62; ++trial) {
            for (int i = count - 1; i > 0; --i) {
                st ^= st << 13;
                st ^= st >> 7;
                st ^= st << 17;
                const int j = (int)(st % (uint64_t)(i + 1));
                std::swap(order[i], order[j]);
            }
            p = first_fit(k, idx, order, W);
            if (p.passes.size() < best.passes.size())
                best = p;
        }
    }
    const size_t slots = std::max<size_t>(1, best.passes.size()) * W;
    rec.assign(slots * 4, -1);
    par.assign(slots * 2, 0.0);
    for (size_t b = 0; b < best.passes.size(); ++b)
        for (size_t q = 0; q < best.passes[b].size(); ++q) {
            const size_t sl = b * W + q;
            const int t = best.passes[b][q].first, o = best.passes[b][q].second;
            for (int r = 0; r < 4; ++r)
                rec[sl * 4 + r] = r < k ? idx[(size_t)t * k + (o ? k - 1 - r : r)] : 0;
            par[sl * 2] = p0[t];
            par[sl * 2 + 1] = p1[t];
        }
}

// Dihedrals grouped by their central bond (j, k): up to three outer atoms i on
// the j side and three l on the k side, every (i, l) combination one term
// (k cos(delta), n), so that one lane computes the shared bond vector, the
// plane normals of each i and each l once and the up to nine torsions from
// them.  Slot record: 8 atoms in roles j, k, i0, i1, i2, l0, l1, l2 (-1: none;
// j = -1: empty slot) and 9 (k cos(delta), n) pairs for (i_a, l_c) at 3 a + c
// (k cos(delta) = 0, n = 1 where no term).  Passes of W slots in which no two
// lanes name the same atom in the same role: a group may be reversed
// (j <-> k, i <-> l) and its outer atoms permuted among their three roles.
// Orders tried: the input order and 63 fixed-seed shuffles; fewest passes
// kept.  Returns the slot count (a multiple of W, 0 without dihedrals).
struct DihGroup {
    int j, k;
    int I[3], L[3];
    int term[3][3];   // dihedral index of (I[a], L[c]) or -1
    int ni, nl;
};

static std::vector<DihGroup> dihedral_groups(const pamd_system& s)
{
    std::vector<DihGroup> g;
    for (int q = 0; q < s.n_dihedrals; ++q) {
        int i = s.dih_idx[4 * q], j = s.dih_idx[4 * q + 1], k = s.dih_idx[4 * q + 2], l = s.dih_idx[4 * q + 3];
        if (j > k) {
            std::swap(i, l);
            std::swap(j, k);
        }
        bool placed = false;
        for (DihGroup& G : g) {
            if (G.j != j || G.k != k)
                continue;
            int a = -1, c = -1;
            for (int u = 0; u < G.ni; ++u)
                if (G.I[u] == i)
                    a = u;
            for (int u = 0; u < G.nl; ++u)
                if (G.L[u] == l)
                    c = u;
            if ((a < 0 && G.ni == 3) || (c < 0 && G.nl == 3) || (a >= 0 && c >= 0 && G.term[a][c] >= 0))
                continue;
            if (a < 0) {
                a = G.ni++;
                G.I[a] = i;
            }
            if (c < 0) {
                c = G.nl++;
                G.L[c] = l;
            }
            G.term[a][c] = q;
            placed = true;
            break;
        }
        if (!placed) {
            DihGroup G;
            G.j = j;
            G.k = k;
            G.ni = G.nl = 1;
            G.I[0] = i;
            G.L[0] = l;
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c)
                    G.term[a][c] = -1;
            G.I[1] = G.I[2] = G.L[1] = G.L[2] = -1;
            G.term[0][0] = q;
            g.push_back(G);
        }
    }
    return g;
}

namespace {
// one placed group: orientation and the role index of each outer atom
struct Placed {
    int grp, flip;
    int ri[3], rl[3];
};
}  // namespace

static std::vector<std::vector<Placed>> pack_groups(const std::vector<DihGroup>& g, const std::vector<int>& order,
                                                    int W)
{
    constexpr int kWords = (PAMD_MAX_ATOMS + 63) / 64;
    struct Used {
        uint64_t bits[8][kWords];
        bool has(int r, int a) const { return (bits[r][a >> 6] >> (a & 63)) & 1u; }
        void set(int r, int a) { bits[r][a >> 6] |= (uint64_t)1 << (a & 63); }
    };
    std::vector<std::vector<Placed>> passes;
    std::vector<Used> used;
    // roles 2.. / 5.. for n outer atoms: first permutation whose roles are free
    auto assign = [](const Used& u, const int* at, int n, int base, int* role) {
        static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        for (const auto& pm : perm) {
            bool ok = true;
            for (int a = 0; a < n && ok; ++a)
                ok = !u.has(base + pm[a], at[a]);
            if (ok) {
                for (int a = 0; a < n; ++a)
                    role[a] = pm[a];
                return true;
            }
        }
        return false;
    };
    for (int gi : order) {
        const DihGroup& G = g[gi];
        bool placed = false;
        for (int flip = 0; flip < 2 && !placed; ++flip) {
            const int j = flip ? G.k : G.j, k = flip ? G.j : G.k;
            const int* I = flip ? G.L : G.I;
            const int* L = flip ? G.I : G.L;
            const int ni = flip ? G.nl : G.ni, nl = flip ? G.ni : G.nl;
            for (size_t b = 0; b < passes.size() && !placed; ++b) {
                if (passes[b].size() >= (size_t)W || used[b].has(0, j) || used[b].has(1, k))
                    continue;
                Placed P{gi, flip, {0, 1, 2}, {0, 1, 2}};
                if (!assign(used[b], I, ni, 2, P.ri) || !assign(used[b], L, nl, 5, P.rl))
                    continue;
                used[b].set(0, j);
                used[b].set(1, k);
                for (int a = 0; a < ni; ++a)
                    used[b].set(2 + P.ri[a], I[a]);
                for (int c = 0; c < nl; ++c)
                    used[b].set(5 + P.rl[c], L[c]);
                passes[b].push_back(P);
                placed = true;
            }
        }
        if (!placed) {
            Used u;
            memset(&u, 0, sizeof(u));
            u.set(0, G.j);
            u.set(1, G.k);
            for (int a = 0; a < G.ni; ++a)
                u.set(2 + a, G.I[a]);
            for (int c = 0; c < G.nl; ++c)
                u.set(5 + c, G.L[c]);
            used.push_back(u);
            passes.push_back({Placed{gi, 0, {0, 1, 2}, {0, 1, 2}}});
        }
    }
    return passes;
}

int pack_dihedral_groups(const pamd_system& s, int W, std::vector<int32_t>* rec, std::vector<double>* par)
{
    if (s.n_dihedrals <= 0) {
        if (rec)
            rec->clear();
        if (par)
            par->clear();
        return 0;
    }
    const std::vector<DihGroup> g = dihedral_groups(s);
    const int ng = (int)g.size();
    std::vector<int> order(ng);
    for (int q = 0; q < ng; ++q)
        order[q] = q;
    std::vector<std::vector<Placed>> best = pack_groups(g, order, W);
    uint64_t st = 0xD1B54A32D192ED03ull ^ (uint64_t)ng;
    for (int trial = 0; trial < 63; ++trial) {
        for (int i = ng - 1; i > 0; --i) {
            st ^= st << 13;
            st ^= st >> 7;
            st ^= st << 17;
            std::swap(order[i], order[(int)(st % (uint64_t)(i + 1))]);
        }
        std::vector<std::vector<Placed>> p = pack_groups(g, order, W);
        if (p.size() < best.size())
            best = std::move(p);
    }
    const int slots = (int)best.size() * W;
    if (rec && par) {
        rec->assign((size_t)slots * 8, -1);
        par->assign((size_t)slots * 45, 0.0);
        for (int q = 0; q < slots; ++q)
            for (int u = 0; u < 9; ++u)
                (*par)[(size_t)q * 45 + 5 * u + 1] = 1.0;
        for (size_t b = 0; b < best.size(); ++b)
            for (size_t q = 0; q < best[b].size(); ++q) {
                const Placed& P = best[b][q];
                const DihGroup& G = g[P.grp];
                const size_t sl = b * W + q;
                int32_t* r = rec->data() + sl * 8;
                double* pp = par->data() + sl * 45;
                r[0] = P.flip ? G.k : G.j;
                r[1] = P.flip ? G.j : G.k;
                const int ni = P.flip ? G.nl : G.ni, nl = P.flip ? G.ni : G.nl;
                for (int a = 0; a < ni; ++a)
                    r[2 + P.ri[a]] = P.flip ? G.L[a] : G.I[a];
                for (int c = 0; c < nl; ++c)
                    r[5 + P.rl[c]] = P.flip ? G.I[c] : G.L[c];
                for (int a = 0; a < ni; ++a)
                    for (int c = 0; c < nl; ++c) {
                        const int t = P.flip ? G.term[c][a] : G.term[a][c];
                        if (t < 0)
                            continue;
                        const int u = 3 * P.ri[a] + P.rl[c];
                        const double kc = s.dih_k[t] * (cos(s.dih_delta[t]) > 0 ? 1.0 : -1.0);   // k cos(delta)
                        const int nm = s.dih_n[t];
                        pp[5 * u] = kc;
                        pp[5 * u + 1] = (double)nm;
                        // kc n U_{n-1}(c) = c0 + c1 c + c2 c^2 for n <= 3 (U_0 = 1, U_1 = 2c,
                        // U_2 = 4c^2 - 1); n > 3 takes the Chebyshev recurrence in the kernel
                        if (nm == 1) {
                            pp[5 * u + 2] = kc;
                        } else if (nm == 2) {
                            pp[5 * u + 3] = 4.0 * kc;
                        } else if (nm == 3) {
                            pp[5 * u + 2] = -3.0 * kc;
                            pp[5 * u + 4] = 12.0 * kc;
                        }
                    }
            }
    }
    return slots;
}

// Angles grouped by their centre atom j: up to four outer atoms, every pair
// (a, c) of them one angle term (k, theta0), so that one lane normalises each
// bond vector once and evaluates the up to six angles from the unit vectors.
// Slot record: 8 ints (j, o0, o1, o2, o3, -1, -1, -1) (-1: no atom; j = -1:
// empty slot) and 6 (k, theta0) pairs for the outer pairs (0,1) (0,2) (0,3)
// (1,2) (1,3) (2,3) (k = 0 where no term).  Passes of W slots with no atom
// twice in one role; outer atoms may be permuted among their four roles.
// Orders tried: the input order and 63 fixed-seed shuffles; fewest passes kept.
struct AngGroup {
    int j, no;
    int o[4];
    int term[4][4];   // angle index of outer pair (a, c), a < c, or -1
    int bond[4];      // bond term j - o[a] evaluated with the group, or -1
};

static int pair_slot(int a, int c)
{
    if (a > c)
        std::swap(a, c);
    static const int tab[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};
    return tab[a][c];
}

static std::vector<AngGroup> angle_groups(const pamd_system& s)
{
    std::vector<AngGroup> g;
    for (int q = 0; q < s.n_angles; ++q) {
        const int i = s.angle_idx[3 * q], j = s.angle_idx[3 * q + 1], k = s.angle_idx[3 * q + 2];
        bool placed = false;
        for (AngGroup& G : g) {
            if (G.j != j)
                continue;
            int a = -1, c = -1;
            for (int u = 0; u < G.no; ++u) {
                if (G.o[u] == i)
                    a = u;
                if (G.o[u] == k)
                    c = u;
            }
            const int need = (a < 0) + (c < 0);
            if (G.no + need > 4 || (a >= 0 && c >= 0 && G.term[a][c] >= 0))
                continue;
            if (a < 0)
                G.o[a = G.no++] = i;
            if (c < 0)
                G.o[c = G.no++] = k;
            G.term[a][c] = G.term[c][a] = q;
            placed = true;
            break;
        }
        if (!placed) {
            AngGroup G;
            G.j = j;
            G.no = 2;
            G.o[0] = i;
            G.o[1] = k;
            G.o[2] = G.o[3] = -1;
            for (int a = 0; a < 4; ++a)
                for (int c = 0; c < 4; ++c)
                    G.term[a][c] = -1;
            G.term[0][1] = G.term[1][0] = q;
            G.bond[0] = G.bond[1] = G.bond[2] = G.bond[3] = -1;
            g.push_back(G);
        }
    }
    // every bond j - a of a group's centre and one of its outer atoms is
    // evaluated with that group (it has the bond vector and its length); each
    // bond term once, the first group and outer role found
    for (int q = 0; q < s.n_bonds; ++q) {
        const int i = s.bond_idx[2 * q], k = s.bond_idx[2 * q + 1];
        bool done = false;
        for (AngGroup& G : g) {
            for (int a = 0; a < G.no && !done; ++a)
                if (G.bond[a] < 0 && ((G.j == i && G.o[a] == k) || (G.j == k && G.o[a] == i))) {
                    G.bond[a] = q;
                    done = true;
                }
            if (done)
                break;
        }
    }
    return g;
}

// bond terms no angle group evaluates (the bond passes): indices and parameters
static void orphan_bonds(const pamd_system& s, std::vector<int32_t>& idx, std::vector<double>& k,
                         std::vector<double>& r0)
{
    std::vector<char> folded(s.n_bonds, 0);
    if (s.n_angles > 0)
        for (const AngGroup& G : angle_groups(s))
            for (int a = 0; a < G.no; ++a)
                if (G.bond[a] >= 0)
                    folded[G.bond[a]] = 1;
    idx.clear();
    k.clear();
    r0.clear();
    for (int q = 0; q < s.n_bonds; ++q)
        if (!folded[q]) {
            idx.push_back(s.bond_idx[2 * q]);
            idx.push_back(s.bond_idx[2 * q + 1]);
            k.push_back(s.bond_k[q]);
            r0.push_back(s.bond_r0[q]);
        }
}

static std::vector<std::vector<std::pair<int, std::array<int, 4>>>> pack_angle_passes(
    const std::vector<AngGroup>& g, const std::vector<int>& order, int W, int nroles)
{
    constexpr int kWords = (PAMD_MAX_ATOMS + 63) / 64;
    struct Used {
        uint64_t bits[5][kWords];
        bool has(int r, int a) const { return (bits[r][a >> 6] >> (a & 63)) & 1u; }
        void set(int r, int a) { bits[r][a >> 6] |= (uint64_t)1 << (a & 63); }
    };
    std::vector<std::vector<std::pair<int, std::array<int, 4>>>> passes;
    std::vector<Used> used;
    for (int gi : order) {
        const AngGroup& G = g[gi];
        bool placed = false;
        for (size_t b = 0; b < passes.size() && !placed; ++b) {
            if (passes[b].size() >= (size_t)W || used[b].has(0, G.j))
                continue;
            std::array<int, 4> perm = {0, 1, 2, 3};
            do {
                bool ok = true;
                for (int a = 0; a < G.no && ok; ++a)
                    ok = perm[a] < nroles && !used[b].has(1 + perm[a], G.o[a]);
                if (ok) {
                    used[b].set(0, G.j);
                    for (int a = 0; a < G.no; ++a)
                        used[b].set(1 + perm[a], G.o[a]);
                    passes[b].push_back({gi, perm});
                    placed = true;
                }
            } while (!placed && std::next_permutation(perm.begin(), perm.end()));
        }
        if (!placed) {
            Used u;
            memset(&u, 0, sizeof(u));
            u.set(0, G.j);
            for (int a = 0; a < G.no; ++a)
                u.set(1 + a, G.o[a]);
            used.push_back(u);
            passes.push_back({{gi, std::array<int, 4>{0, 1, 2, 3}}});
        }
    }
    return passes;
}

// Angle groups packed in two classes: groups with four outer atoms (six
// angles) first, then groups with at most three (three angles, outer roles
// 0..2), so the kernel runs the cheaper three-angle body on the second
// class.  *n6 (optional) = slots of the first class (a multiple of W).
int pack_angle_groups(const pamd_system& s, int W, std::vector<int32_t>* rec, std::vector<double>* par,
                      int* n6 = nullptr)
{
    if (s.n_angles <= 0) {
        if (rec)
            rec->clear();
        if (par)
            par->clear();
        if (n6)
            *n6 = 0;
        return 0;
    }
    const std::vector<AngGroup> g = angle_groups(s);
    std::vector<std::vector<std::pair<int, std::array<int, 4>>>> best;
    size_t passes6 = 0;
    for (int cls = 0; cls < 2; ++cls) {
        std::vector<int> order;
        for (int q = 0; q < (int)g.size(); ++q)
            if ((g[q].no == 4) == (cls == 0))
                order.push_back(q);
        if (order.empty())
            continue;
        const int nroles = cls == 0 ? 4 : 3;
        auto cbest = pack_angle_passes(g, order, W, nroles);
        uint64_t st = 0xA0761D6478BD642Full ^ (uint64_t)(order.size() + 977 * cls);
        for (int trial = 0; trial < 63; ++trial) {
            for (int i = (int)order.size() - 1; i > 0; --i) {
                st ^= st << 13;
                st ^= st >> 7;
                st ^= st << 17;
                std::swap(order[i], order[(int)(st % (uint64_t)(i + 1))]);
            }
            auto p = pack_angle_passes(g, order, W, nroles);
            if (p.size() < cbest.size())
                cbest = std::move(p);
        }
        if (cls == 0)
            passes6 = cbest.size();
        for (auto& pass : cbest)
            best.push_back(std::move(pass));
    }
    if (n6)
        *n6 = (int)passes6 * W;
    const int slots = (int)best.size() * W;
    if (rec && par) {
        rec->assign((size_t)slots * 8, -1);
        par->assign((size_t)slots * kAngPar, 0.0);
        for (size_t b = 0; b < best.size(); ++b)
            for (size_t q = 0; q < best[b].size(); ++q) {
                const AngGroup& G = g[best[b][q].first];
                const std::array<int, 4>& perm = best[b][q].second;
                const size_t sl = b * W + q;
                int32_t* r = rec->data() + sl * 8;
                double* pp = par->data() + sl * kAngPar;
                r[0] = G.j;
                for (int a = 0; a < G.no; ++a) {
                    r[1 + perm[a]] = G.o[a];
                    if (G.bond[a] >= 0) {
                        pp[12 + 2 * perm[a]] = s.bond_k[G.bond[a]];
                        pp[13 + 2 * perm[a]] = s.bond_r0[G.bond[a]];
                    }
                }
                for (int a = 0; a < G.no; ++a)
                    for (int c = a + 1; c < G.no; ++c) {
                        const int t = G.term[a][c];
                        if (t < 0)
                            continue;
                        const int u = pair_slot(perm[a], perm[c]);
                        pp[2 * u] = s.angle_k[t];
                        pp[2 * u + 1] = s.angle_theta0[t];
                    }
            }
    }
    return slots;
}

// Pair coefficients in the order the MD kernel walks its tiles: for block J,
// the diagonal block (rotations k = 1..8; k = 8 only on lanes 0..7), then for
// k = 0..15 the blocks I < J.  Lane l of step (I, J, k) pairs atom 16 I + l
// with atom 16 J + ((l - k) mod 16).
void build_tables(const pamd_system& s, HostTables& t, int wide, int lj_rows)
{
    const int n = s.n_atoms;
    t.n = n;
    t.wide = wide;
    t.nslot = nslot_of(n);
    t.npad = npad_of(n, wide);
    const std::vector<int> dist = graph_distance(n, s.n_bonds, s.bond_idx);
    const int steps = wide ? 0 : tile_steps(t.nslot);
    const int W = wide ? kWide : kRow;
    t.ab.assign((size_t)steps * 16 * 2, 0.0);
    t.c.assign((size_t)steps * 16, 0.0);
    auto coef = [&](int st, int l, int i, int j) {
        if (i >= n || j >= n || i == j)
            return;
        const int g = dist[(size_t)i * n + j];
        if (g <= 2)
            return;   // 1-2 and 1-3 pairs are excluded
        const double slj = (g == 3) ? s.scale14_lj : 1.0;
        const double sc = (g == 3) ? s.scale14_coul : 1.0;
        const double sig = 0.5 * (s.sigma[i] + s.sigma[j]);
        const double eps = sqrt(s.epsilon[i] * s.epsilon[j]);
        const double s6 = pow(sig, 6.0);
        const double c6 = 4.0 * eps * s6, c12 = 4.0 * eps * s6 * s6;
        const double qq = s.coulomb_k * s.charge[i] * s.charge[j] * sc;
        t.ab[((size_t)st * 16 + l) * 2] = 12.0 * c12 * slj;
        t.ab[((size_t)st * 16 + l) * 2 + 1] = -6.0 * c6 * slj;
        t.c[(size_t)st * 16 + l] = (s.dielectric == PAMD_DIELECTRIC_4R) ? 2.0 * qq / 4.0 : qq;
    };
    int st = 0;
    for (int J = 0; J < (wide ? 0 : t.nslot); ++J) {
        for (int k = 1; k <= 8; ++k, ++st)
            for (int l = 0; l < 16; ++l)
                if (!(k == 8 && l >= 8))
                    coef(st, l, 16 * J + l, 16 * J + ((l - k) & 15));
        for (int k = 0; k < 16; ++k)
            for (int I = 0; I < J; ++I, ++st)
                for (int l = 0; l < 16; ++l)
                    coef(st, l, 16 * I + l, 16 * J + ((l - k) & 15));
    }
    if (wide) {
        // per-atom Coulomb factor (Coulomb factor of a pair = qs_i qs_j) and
        // LJ class; the class table holds 12 c12 and -6 c6 of every class
        // pair, combined as for the per-pair tables above (the padding class
        // stays zero; pamd_query_sizes has checked the class count)
        const double cf = (s.dielectric == PAMD_DIELECTRIC_4R) ? 0.5 : 1.0;
        t.nchunk = (n + 31) / 32;
        t.atomp.assign((size_t)n * 2, 0.0);
        t.pmask.assign((size_t)n * t.nchunk * 2, 0u);
        std::vector<int> cls;
        lj_classes(s, &cls);
        const int ljs = lj_stride_of(lj_rows);
        t.lj.assign((size_t)lj_rows * ljs * 2, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double sig = 0.5 * (s.sigma[i] + s.sigma[j]);
                const double eps = sqrt(s.epsilon[i] * s.epsilon[j]);
                const double s6 = pow(sig, 6.0);
                const size_t e = ((size_t)cls[i] * ljs + cls[j]) * 2;
                t.lj[e] = 12.0 * 4.0 * eps * s6 * s6;
                t.lj[e + 1] = -6.0 * 4.0 * eps * s6;
            }
        for (int i = 0; i < n; ++i) {
            t.atomp[2 * i] = s.charge[i] * sqrt(s.coulomb_k * cf);
            t.atomp[2 * i + 1] = cls[i];
            for (int j = 0; j < n; ++j) {
                const int g = dist[(size_t)i * n + j];
                const size_t w = ((size_t)i * t.nchunk + j / 32) * 2;
                if (i == j || g <= 2)
                    t.pmask[w] |= 1u << (j & 31);
                else if (g == 3)
                    t.pmask[w + 1] |= 1u << (j & 31);
            }
        }
        // rotation steps of the nonbonded ring that meet an excluded or 1-4
        // pair on some lane: at step k own atom 64 s + l meets partner
        // 64 t + (l + k) mod 64; the same-slot ring also keeps its k = 32 step
        // (the pair seen from both lanes) on the masked path
        t.stepmask.assign((size_t)kWideSlots * kWideSlots, 0ull);
        const int nsl = (n + kWide - 1) / kWide;
        for (int tt = 0; tt < nsl; ++tt)
            for (int ss = 0; ss <= tt; ++ss) {
                uint64_t m = ss == tt ? (1ull | (1ull << 32)) : 0ull;
                for (int k = 0; k < kWide; ++k)
                    for (int l = 0; l < kWide && !((m >> k) & 1ull); ++l) {
                        const int a = kWide * ss + l, j = kWide * tt + (l + k) % kWide;
                        if (a < n && j < n && (a == j || dist[(size_t)a * n + j] <= 3))
                            m |= 1ull << k;
                    }
                t.stepmask[(size_t)tt * kWideSlots + ss] = m;
            }
    }
    std::vector<int32_t> bi;
    std::vector<double> bk, br;
    orphan_bonds(s, bi, bk, br);
    pack_terms((int)bk.size(), 2, bi.data(), bk.data(), br.data(), t.bidx, t.bpar, W);
    pack_angle_groups(s, W, &t.aidx, &t.apar, &t.n6);
    pack_dihedral_groups(s, W, &t.didx, &t.dpar);
    t.mass.assign(t.npad, 0.0);
    t.mtot = 0;
    for (int a = 0; a < n; ++a) {
        t.mass[a] = s.mass[a];
        t.mtot += s.mass[a];
    }
    t.x_init.assign(s.x_init, s.x_init + 3 * n);
}

template <typename real>
void carve(Carver& st, Carver& wk, const pamd_system& s, const pamd_params& p, int run, RunDev<real>& d, int wide)
{
    const int n = s.n_atoms;
    const int nslot = nslot_of(n);
    const int npad = npad_of(n, wide);
    const int64_t Rc = p.R_cap;
    const int steps = wide ? 0 : tile_steps(nslot);
    const int W = wide ? kWide : kRow;
    const int nchunk = (n + 31) / 32;
    for (int b = 0; b < 2; ++b)
        d.slab[b] = st.take<real>((size_t)Rc * 6 * npad);
    for (int b = 0; b < 2; ++b)
        d.epot[b] = st.take<double>(Rc);
    for (int b = 0; b < 2; ++b)
        d.ekin[b] = st.take<double>(Rc);
    for (int b = 0; b < 2; ++b)
        d.anc[b] = st.take<int32_t>(Rc);
    d.ctl = wk.take<RunCtl>(1);
    d.counts = wk.take<int32_t>(Rc);
    d.src_of = wk.take<int32_t>(Rc);
    d.cdf = wk.take<double>(Rc);
    d.part = wk.take<double>(part_doubles(Rc));
    d.cpart = wk.take<int64_t>(cpart_count(Rc));
    d.fam = wk.take<uint8_t>(p.R_target);
    d.nb_ab = wk.take<real>((size_t)steps * 32);
    d.nb_c = wk.take<real>((size_t)steps * 16);
    // packed term slots (passes of W lanes)
    std::vector<int32_t> rec;
    std::vector<double> par;
    std::vector<double> zeros(std::max({s.n_bonds, s.n_angles, s.n_dihedrals, 1}), 0.0);
    std::vector<int32_t> bi;
    std::vector<double> bk, br;
    orphan_bonds(s, bi, bk, br);
    pack_terms((int)bk.size(), 2, bi.data(), zeros.data(), zeros.data(), rec, par, W);
    const int nb_slots = (int)(rec.size() / 4);
    int na6 = 0;
    const int na_slots = std::max(pack_angle_groups(s, W, nullptr, nullptr, &na6), 1);
    const int nd_slots = std::max(pack_dihedral_groups(s, W, nullptr, nullptr), 1);
    d.bidx = wk.take<int4>(nb_slots);
    d.bpar = wk.take<real>((size_t)nb_slots * 2);
    d.agrp = wk.take<int4>((size_t)na_slots * 2);
    d.agpar = wk.take<real>((size_t)na_slots * kAngPar);
    d.dgrp = wk.take<int4>((size_t)nd_slots * 2);
    d.dgpar = wk.take<real>((size_t)nd_slots * 45);
    d.mass = wk.take<double>(npad);
    d.x_init = wk.take<double>((size_t)3 * n);
    d.sched = wk.take<double>(kMaxSched);
    d.n_sched = 0;
    d.dbg = wk.take<double>((size_t)PAMD_FORCE_CHUNK * npad * 4);
    d.obs = wk.take<pamd_obs>(1);
    d.unif = nullptr;
    d.n = n;
    d.npad = npad;
    d.nslot = nslot;
    d.nb = !bk.empty() ? nb_slots : 0;
    d.nag = s.n_angles > 0 ? na_slots : 0;
    d.nag6 = s.n_angles > 0 ? na6 : 0;
    d.dih_general = 0;
    for (int t = 0; t < s.n_dihedrals; ++t)
        if (s.dih_n[t] > 3)
            d.dih_general = 1;
    d.ng = s.n_dihedrals > 0 ? nd_slots : 0;
    d.R_target = p.R_target;
    d.R_cap = Rc;
    d.kB = s.kB;
    d.dt = p.dt;
    d.T0 = p.T0;
    d.V_target = p.V_target > 0 ? p.V_target : 0.1;
    d.T_final = p.T_final > 0 ? p.T_final : p.T0;
    d.thermostat = p.thermostat;
    d.p24 = p.thermostat == PAMD_THERMOSTAT_ANDERSEN ? (uint32_t)llround((1.0 - exp(-p.nu * p.dt)) * 16777216.0)
                                                     : 0u;
    d.lc1 = exp(-p.nu * p.dt);
    d.lc2 = sqrt(1.0 - d.lc1 * d.lc1);
    d.key0 = (uint32_t)(p.seed & 0xFFFFFFFFu);
    d.key1 = (uint32_t)(p.seed >> 32) + (uint32_t)run;
    d.dielectric = s.dielectric;
    d.resampling = p.resampling;
    d.wide = wide;
    d.nchunk = wide ? nchunk : 0;
    d.apar2 = wide ? wk.take<float2>(n) : nullptr;
    d.ljtab = wide ? wk.take<float2>((size_t)kLjClasses * kLjStride) : nullptr;
    d.pmask = wide ? wk.take<uint2>((size_t)n * nchunk) : nullptr;
    d.stepmask = wide ? wk.take<uint64_t>((size_t)kWideSlots * kWideSlots) : nullptr;
    d.s14lj = (float)s.scale14_lj;
    d.s14c = (float)s.scale14_coul;
}

template <typename real>
hipError_t upload(const RunDev<real>& d, const HostTables& t, hipStream_t s)
{
    auto up = [&](const void* dst, const std::vector<double>& src) -> hipError_t {
        std::vector<real> tmp(src.begin(), src.end());
        hipError_t e = hipMemcpyAsync((void*)dst, tmp.data(), tmp.size() * sizeof(real), hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return e;
        return hipStreamSynchronize(s);
    };
    auto upi = [&](const void* dst, const std::vector<int32_t>& src) -> hipError_t {
        hipError_t e = hipMemcpyAsync((void*)dst, src.data(), src.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return e;
        return hipStreamSynchronize(s);
    };
    auto upd = [&](const void* dst, const std::vector<double>& src) -> hipError_t {
        hipError_t e = hipMemcpyAsync((void*)dst, src.data(), src.size() * sizeof(double), hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return e;
        return hipStreamSynchronize(s);
    };
    hipError_t e;
    if (!t.ab.empty() && (e = up(d.nb_ab, t.ab)) != hipSuccess) return e;
    if (!t.c.empty() && (e = up(d.nb_c, t.c)) != hipSuccess) return e;
    if (t.wide) {
        std::vector<float> ap(t.atomp.begin(), t.atomp.end());
        if ((e = hipMemcpyAsync((void*)d.apar2, ap.data(), ap.size() * sizeof(float), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            return e;
        std::vector<float> lj(t.lj.begin(), t.lj.end());
        if ((e = hipMemcpyAsync((void*)d.ljtab, lj.data(), lj.size() * sizeof(float), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            return e;
        if ((e = hipMemcpyAsync((void*)d.pmask, t.pmask.data(), t.pmask.size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
        if ((e = hipMemcpyAsync((void*)d.stepmask, t.stepmask.data(), t.stepmask.size() * sizeof(uint64_t),
                                hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    }
    if ((e = upi(d.bidx, t.bidx)) != hipSuccess) return e;
    if ((e = up(d.bpar, t.bpar)) != hipSuccess) return e;
    if (!t.aidx.empty() && (e = upi(d.agrp, t.aidx)) != hipSuccess) return e;
    if (!t.apar.empty() && (e = up(d.agpar, t.apar)) != hipSuccess) return e;
    if (!t.didx.empty() && (e = upi(d.dgrp, t.didx)) != hipSuccess) return e;
    if (!t.dpar.empty() && (e = up(d.dgpar, t.dpar)) != hipSuccess) return e;
    if ((e = upd(d.mass, t.mass)) != hipSuccess) return e;
    if ((e = upd(d.x_init, t.x_init)) != hipSuccess) return e;
    return hipSuccess;
}

pamd_status layout(const pamd_system* sys, int32_t n_runs, const pamd_params* p, void* d_state, void* d_work,
                   std::vector<Run>* runs, size_t* sb, size_t* wb, pamd_ctx* c)
{
    Carver st(d_state), wk(d_work);
    const int fp32 = p[0].precision == PAMD_FP32;
    int wide = 0;
    for (int r = 0; r < n_runs; ++r) {
        if (fp32) {
            RunDev<float> d{};
            const int w = run_is_wide(sys, p, n_runs, r);
            wide |= w;
            carve<float>(st, wk, sys[r], p[r], r, d, w);
            if (runs)
                (*runs)[r].f = d;
        } else {
            RunDev<double> d{};
            carve<double>(st, wk, sys[r], p[r], r, d, 0);
            if (runs)
                (*runs)[r].d = d;
        }
    }
    if (wide) {
        // descriptors, run order and work counter of the batched launch
        RunDev<float>* dr = wk.take<RunDev<float>>(n_runs);
        int32_t* order = wk.take<int32_t>(n_runs);
        int32_t* counter = wk.take<int32_t>(1);
        if (c) {
            c->wide = 1;
            c->d_runs = dr;
            c->d_order = order;
            c->d_counter = counter;
        }
    }
    *sb = (st.off + kAlign - 1) / kAlign * kAlign;
    *wb = (wk.off + kAlign - 1) / kAlign * kAlign;
    return PAMD_OK;
}

template <typename real>
RunDev<real>& dev(Run& r);
template <>
RunDev<float>& dev<float>(Run& r) { return r.f; }
template <>
RunDev<double>& dev<double>(Run& r) { return r.d; }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

pamd_status check_ctx(pamd_ctx* c)
{
    if (!c)
        return PAMD_ERR_ARG;
    if (c->failed)
        return fail(c, PAMD_ERR_STATE, "context failed earlier: " + c->err);
    return PAMD_OK;
}

template <typename real>
pamd_status read_ctl(pamd_ctx* c, Run& run, RunCtl* ctl, hipStream_t s)
{
    HIPCHK(c, hipMemcpyAsync(ctl, dev<real>(run).ctl, sizeof(RunCtl), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return PAMD_OK;
}

pamd_status surface_device_error(pamd_ctx* c, int code)
{
    if (code == 0)
        return PAMD_OK;
    const char* what = code == PAMD_ERR_CAPACITY   ? "resampled population over capacity (or extinct)"
                       : code == PAMD_ERR_NONFINITE ? "non-finite potential energy"
                       : code == PAMD_ERR_INTERNAL  ? "an index check of the bounds-checked build failed"
                                                    : "device error";
    return fail(c, code, what);
}

}  // namespace

// Entry points: declared extern "C" in pamd.h, so these definitions have C linkage.

pamd_status pamd_query_sizes(const pamd_system* sys, int32_t n_runs, const pamd_params* p, size_t* state_bytes,
                             size_t* work_bytes)
{
    if (!sys || !p || !state_bytes || !work_bytes || n_runs < 1)
        return PAMD_ERR_ARG;
    const int fp32 = p[0].precision == PAMD_FP32;
    for (int r = 0; r < n_runs; ++r) {
        if (p[r].precision != p[0].precision || p[r].thermostat != p[0].thermostat)
            return PAMD_ERR_ARG;
        pamd_status st = validate(nullptr, sys[r], p[r], fp32);
        if (st != PAMD_OK)
            return st;
        // the wide kernels read LJ pair coefficients from a class table
        if (run_is_wide(sys, p, n_runs, r) && lj_classes(sys[r], nullptr) > kLjClasses - 1)
            return PAMD_ERR_ARG;
    }
    return layout(sys, n_runs, p, nullptr, nullptr, nullptr, state_bytes, work_bytes, nullptr);
}

template <typename real>
static pamd_status init_runs(pamd_ctx* c, const pamd_system* sys, hipStream_t s)
{
    for (int r = 0; r < c->n_runs; ++r) {
        Run& run = c->runs[r];
        build_tables(sys[r], run.tab, c->fp32 ? run.f.wide : 0, c->lj_rows);
        if (c->fp32 && run.f.wide) {
            run.f.lj_stride = lj_stride_of(c->lj_rows);
            run.f.lj_pad = c->lj_rows - 1;
        }
        run.mtot = run.tab.mtot;
        HIPCHK(c, upload<real>(dev<real>(run), run.tab, s));
        HIPCHK(c, launch_init(dev<real>(run), s));
    }
    if (c->wide) {
        // the batched launch's descriptors and its largest-first order of the wide runs
        std::vector<RunDev<float>> rd(c->n_runs);
        std::vector<int32_t> order;
        for (int r = 0; r < c->n_runs; ++r) {
            rd[r] = c->runs[r].f;
            if (c->runs[r].f.wide)
                order.push_back(r);
        }
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return sys[a].n_atoms > sys[b].n_atoms; });
        c->n_wide = (int)order.size();
        HIPCHK(c, hipMemcpyAsync(c->d_runs, rd.data(), rd.size() * sizeof(RunDev<float>), hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(c->d_order, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemsetAsync(c->d_counter, 0, sizeof(int32_t), s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    return PAMD_OK;
}

pamd_status pamd_init(const pamd_system* sys, int32_t n_runs, const pamd_params* p, void* d_state,
                      size_t state_bytes, void* d_work, size_t work_bytes, void* stream, pamd_ctx** out)
{
    TraceRange trace_range("pamd_init");
    if (!out)
        return PAMD_ERR_ARG;
    *out = nullptr;
    if (!sys || !p || n_runs < 1 || !d_state || !d_work)
        return PAMD_ERR_ARG;
    if (((uintptr_t)d_state % kAlign) || ((uintptr_t)d_work % kAlign))
        return PAMD_ERR_ARG;
    size_t sb = 0, wb = 0;
    pamd_status st = pamd_query_sizes(sys, n_runs, p, &sb, &wb);
    if (st != PAMD_OK)
        return st;
    if (state_bytes < sb || work_bytes < wb)
        return PAMD_ERR_ARG;
    pamd_ctx* c = new pamd_ctx();
    *out = c;
    c->n_runs = n_runs;
    c->fp32 = p[0].precision == PAMD_FP32;
    c->runs.resize(n_runs);
    layout(sys, n_runs, p, d_state, d_work, &c->runs, &sb, &wb, c);
    hipStream_t s = as_stream(stream);

    int dev_id = 0;
    HIPCHK(c, hipGetDevice(&dev_id));
    HIPCHK(c, hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, dev_id));
    int max_lds = 0;
    HIPCHK(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev_id));

    // launch shapes.  Register-tile runs: the largest workgroup (<= 16 waves)
    // whose LDS fits, shared by those runs.  Wide runs: one replica per
    // wavefront, at most 4 waves (256 threads) per workgroup.  Both with
    // enough resident blocks to fill every CU.
    int tn_max = 0, ts_max = 0, wn_max = 0, n_tile = 0;
    for (int r = 0; r < n_runs; ++r) {
        if (c->fp32 && c->runs[r].f.wide) {
            wn_max = std::max(wn_max, sys[r].n_atoms);
        } else {
            ++n_tile;
            tn_max = std::max(tn_max, sys[r].n_atoms);
            ts_max = std::max(ts_max, nslot_of(sys[r].n_atoms));
        }
    }
    c->nmax = wn_max;
    c->diel = sys[0].dielectric;
    for (int r = 1; r < n_runs; ++r)
        if (c->wide && sys[r].dielectric != sys[0].dielectric)
            return fail(c, PAMD_ERR_ARG, "runs of a context with a batched launch must share the dielectric model");
    if (c->wide) {
        // LJ class tables shaped for the largest class count of the wide runs
        int lj_max = 1;
        for (int r = 0; r < n_runs; ++r)
            if (c->runs[r].f.wide)
                lj_max = std::max(lj_max, lj_classes(sys[r], nullptr));
        c->lj_rows = lj_max + 1;
        const int ljsz = c->lj_rows * lj_stride_of(c->lj_rows);
        int waves = p[0].wide_waves_per_block;
        if (waves == 0)
            waves = 4;
        while (waves > 1 && wide_lds_bytes(wn_max, waves, ljsz) > (size_t)max_lds)
            --waves;
        int bpc = 0;
        HIPCHK(c, wide_setup(c->diel, wn_max, waves, ljsz, &bpc));
        if (bpc < 1)
            return fail(c, PAMD_ERR_ARG, "batched MD kernel cannot be resident with this launch shape");
        c->wide_waves = waves;
        c->wide_blocks = c->n_cu * bpc;
        c->wide_lds = wide_lds_bytes(wn_max, waves, ljsz);
    }
    if (n_tile > 0) {
        int waves = p[0].waves_per_block;
        if (waves == 0) {
            waves = 16;
            while (waves > 1 && md_lds(c->fp32, ts_max, tn_max, waves) > (size_t)max_lds)
                --waves;
        }
        c->tile_lds = md_lds(c->fp32, ts_max, tn_max, waves);
        if (c->tile_lds > (size_t)max_lds)
            return fail(c, PAMD_ERR_ARG, "system too large for the LDS of one workgroup");
        int bpc = 0;
        HIPCHK(c, md_occupancy(c->fp32, ts_max, sys[0].dielectric, tn_max, waves, &bpc));
        if (bpc < 1)
            return fail(c, PAMD_ERR_ARG, "MD kernel cannot be resident with this launch shape");
        c->tile_waves = waves;
        c->tile_blocks = c->n_cu * bpc;
    }
    for (int r = 0; r < n_runs; ++r) {
        const int w = c->fp32 && c->runs[r].f.wide;
        c->runs[r].f.waves_per_block = w ? c->wide_waves : c->tile_waves;
        c->runs[r].d.waves_per_block = c->tile_waves;
        c->runs[r].nu = p[r].nu;
    }
    // side streams (default priority) when register-tile launches can overlap
    if (n_tile >= 2) {
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        for (int k = 0; k < std::min(n_tile, pamd_ctx::kSide); ++k) {
            HIPCHK(c, hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking));
            HIPCHK(c, hipEventCreateWithFlags(&c->ev_join[k], hipEventDisableTiming));
            c->n_side = k + 1;
        }
    }
    return c->fp32 ? init_runs<float>(c, sys, s) : init_runs<double>(c, sys, s);
}

// F_NN at the current positions of every replica of `run` into run.mts.fnn
static pamd_status nn_force(pamd_ctx* c, Run& run, hipStream_t s)
{
    const RunDev<float>& d = run.f;
    nn::ConfIO io{};
    io.xbase[0] = d.slab[0];
    io.xbase[1] = d.slab[1];
    io.fout = run.mts.fnn.as<float>();
    io.ctl = d.ctl;
    io.xs_conf = 6 * (int64_t)d.npad;
    io.xs_comp = d.npad;
    io.xs_atom = 1;
    io.fs_conf = 3 * (int64_t)d.npad;
    io.fs_comp = d.npad;
    io.fs_atom = 1;
    const pamd_nn* nn = c->nn;
    HIPCHK(c, nn::launch_features(nn->topo, io, d.R_cap, nullptr, run.mts.G.as<uint16_t>(), s));
    HIPCHK(c, nn::launch_mlp(nn->w, run.mts.G.as<uint16_t>(), run.mts.gG.as<uint16_t>(), run.mts.e.as<float>(), d.ctl,
                             d.R_cap * d.n, d.n, s));
    HIPCHK(c, nn::launch_force(nn->topo, io, d.R_cap, run.mts.gG.as<uint16_t>(), run.mts.e.as<float>(), nullptr, s));
    return PAMD_OK;
}

// n_steps / M r-RESPA outer steps of `run` (M = c->mts_ratio), then the
// exact potential energies.  The last inner half kick, both outer impulses,
// the collisions and the next step's first drift all act at the same
// positions and share one k_respa pass.
static pamd_status respa_steps(pamd_ctx* c, Run& run, int n_steps, hipStream_t s)
{
    const RunDev<float>& d = run.f;
    const int M = c->mts_ratio;
    const int n_outer = n_steps / M;
    const double Dt = M * d.dt;
    const uint32_t p24 = (uint32_t)llround((1.0 - exp(-run.nu * Dt)) * 16777216.0);
    const float* fnn = run.mts.fnn.as<float>();
    pamd_status st = PAMD_OK;
    HIPCHK(c, launch_md_begin(d, s));
    if (n_outer > 0) {
        if ((st = nn_force(c, run, s)) != PAMD_OK)
            return st;
        HIPCHK(c, launch_respa(d, fnn, kRespaOuterStart | kRespaDrift, 0, Dt, p24, c->tile_blocks, c->tile_waves, s));
        for (int o = 0; o < n_outer; ++o) {
            for (int q = 0; q < M; ++q) {
                if ((st = nn_force(c, run, s)) != PAMD_OK)
                    return st;
                if (q < M - 1)
                    HIPCHK(c, launch_respa(d, fnn, kRespaInnerKick | kRespaDrift, 0, Dt, p24, c->tile_blocks, c->tile_waves, s));
            }
            int ops = kRespaInnerKick | kRespaOuterEnd | kRespaCollide;
            if (o < n_outer - 1)
                ops |= kRespaOuterStart | kRespaDrift;
            HIPCHK(c, launch_respa(d, fnn, ops, (uint32_t)(o * M), Dt, p24, c->tile_blocks, c->tile_waves, s));
        }
    }
    HIPCHK(c, launch_energy(d, c->tile_blocks, c->tile_waves, s));
    HIPCHK(c, launch_md_finalize(d, n_steps, s));
    return PAMD_OK;
}

// workgroups of a register-tile launch of `run`.  Alone, the persistent launch
// takes the whole chip's grid: a small population's work items then land on
// waves of every CU, about one per SIMD, the fastest spread for a
// latency-bound launch.  Next to other register-tile launches on side streams
// it takes no more workgroups than its R_cap / 4 items fill, so the launches
// share the chip instead of each holding every CU.
static int tile_launch_blocks(const pamd_ctx* c, int64_t R_cap)
{
    if (c->n_side == 0)
        return c->tile_blocks;
    const int64_t per_block = (int64_t)kRowsPerWave * c->tile_waves;
    return (int)std::min<int64_t>(c->tile_blocks, (R_cap + per_block - 1) / per_block);
}

// PAMD step 3 of one register-tile run on stream t
template <typename real>
static pamd_status enqueue_tile_md(pamd_ctx* c, const RunDev<real>& d, int n_steps, hipStream_t t)
{
    const int blocks = tile_launch_blocks(c, d.R_cap);
    HIPCHK(c, launch_md_begin(d, t));
    HIPCHK(c, launch_md(d, n_steps, blocks, c->tile_waves, t));
    HIPCHK(c, launch_energy(d, blocks, c->tile_waves, t));
    HIPCHK(c, launch_md_finalize(d, n_steps, t));
    return PAMD_OK;
}

pamd_status pamd_md_steps(pamd_ctx* c, int32_t n_steps, void* stream)
{
    TraceRange trace_range("pamd_md_steps");
    pamd_status st = check_ctx(c);
    if (st != PAMD_OK)
        return st;
    if (n_steps < 0)
        return fail(c, PAMD_ERR_ARG, "n_steps < 0");
    c->have_energy = 1;
    hipStream_t s = as_stream(stream);
    if (c->n_side > 0 && !(c->nn && n_steps > 0)) {
        // fork: the register-tile runs round robin over the side streams, the
        // wide launch on `s` next to them, then every side stream joined back
        HIPCHK(c, hipEventRecord(c->ev_fork, s));
        int used = 0, k = 0;
        for (auto& run : c->runs) {
            if (c->fp32 && run.f.wide)
                continue;
            hipStream_t t = c->side[k];
            if (k >= used) {
                HIPCHK(c, hipStreamWaitEvent(t, c->ev_fork, 0));
                used = k + 1;
            }
            st = c->fp32 ? enqueue_tile_md(c, run.f, n_steps, t) : enqueue_tile_md(c, run.d, n_steps, t);
            if (st != PAMD_OK)
                return st;
            k = (k + 1) % c->n_side;
        }
        if (c->wide)
            HIPCHK(c, launch_md_wide(c->d_runs, c->d_order, c->n_wide, c->d_counter, c->nmax, n_steps, c->diel,
                                     c->runs[0].f.thermostat == PAMD_THERMOSTAT_LANGEVIN,
                                     c->lj_rows * lj_stride_of(c->lj_rows), c->wide_blocks, c->wide_waves, s));
        for (int q = 0; q < used; ++q) {
            HIPCHK(c, hipEventRecord(c->ev_join[q], c->side[q]));
            HIPCHK(c, hipStreamWaitEvent(s, c->ev_join[q], 0));
        }
        return PAMD_OK;
    }
    if (c->wide)
        HIPCHK(c, launch_md_wide(c->d_runs, c->d_order, c->n_wide, c->d_counter, c->nmax, n_steps, c->diel,
                                 c->runs[0].f.thermostat == PAMD_THERMOSTAT_LANGEVIN,
                                 c->lj_rows * lj_stride_of(c->lj_rows), c->wide_blocks, c->wide_waves, s));
    if (c->nn && n_steps > 0) {
        if (n_steps % c->mts_ratio != 0)
            return fail(c, PAMD_ERR_ARG, "n_steps must be a multiple of the r-RESPA outer ratio");
        for (auto& run : c->runs) {
            st = respa_steps(c, run, n_steps, s);
            if (st != PAMD_OK)
                return st;
        }
        return PAMD_OK;
    }
    for (auto& run : c->runs) {
        if (c->fp32 && run.f.wide)
            continue;   // advanced by the batched launch above
        st = c->fp32 ? enqueue_tile_md(c, run.f, n_steps, s) : enqueue_tile_md(c, run.d, n_steps, s);
        if (st != PAMD_OK)
            return st;
    }
    return PAMD_OK;
}

pamd_status pamd_resample(pamd_ctx* c, const double* T_next, const double* d_uniforms, void* stream)
{
    TraceRange trace_range("pamd_resample");
    pamd_status st = check_ctx(c);
    if (st != PAMD_OK)
        return st;
    if (!c->have_energy) {
        // call-order error: the context stays usable
        c->err = "resample before any MD step: the population has no energies yet";
        return PAMD_ERR_STATE;
    }
    hipStream_t s = as_stream(stream);
    for (int r = 0; r < c->n_runs; ++r) {
        Run& run = c->runs[r];
        const double Treq = T_next ? T_next[r] : 0.0;
        if (c->fp32) {
            RunDev<float> d = run.f;
            d.unif = d_uniforms ? d_uniforms + (size_t)r * d.R_cap : nullptr;
            HIPCHK(c, launch_resample(d, Treq, run.mtot, s));
        } else {
            RunDev<double> d = run.d;
            d.unif = d_uniforms ? d_uniforms + (size_t)r * d.R_cap : nullptr;
            HIPCHK(c, launch_resample(d, Treq, run.mtot, s));
        }
    }
    return PAMD_OK;
}

pamd_status pamd_observables(pamd_ctx* c, pamd_obs* out, void* stream)
{
    TraceRange trace_range("pamd_observables");
    pamd_status st = check_ctx(c);
    if (st != PAMD_OK)
        return st;
    if (!out)
        return fail(c, PAMD_ERR_ARG, "null output");
    hipStream_t s = as_stream(stream);
    for (int r = 0; r < c->n_runs; ++r) {
        Run& run = c->runs[r];
        void* obs = c->fp32 ? run.f.obs : run.d.obs;
        if (c->fp32)
            HIPCHK(c, launch_observables(run.f, s));
        else
            HIPCHK(c, launch_observables(run.d, s));
        HIPCHK(c, hipMemcpyAsync(&out[r], obs, sizeof(pamd_obs), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    for (int r = 0; r < c->n_runs; ++r)
        if (out[r].error)
            return surface_device_error(c, out[r].error);
    return PAMD_OK;
}

template <typename real>
static pamd_status get_forces_t(pamd_ctx* c, Run& run, int64_t r0, int32_t count, double* F, double* E,
                                hipStream_t s)
{
    RunCtl ctl;
    pamd_status st = read_ctl<real>(c, run, &ctl, s);
    if (st != PAMD_OK)
        return st;
    if (ctl.error)
        return surface_device_error(c, ctl.error);
    if (r0 < 0 || count < 1 || count > PAMD_FORCE_CHUNK || r0 + count > ctl.R_cur)
        return fail(c, PAMD_ERR_ARG, "replica range outside the population or chunk");
    RunDev<real>& d = dev<real>(run);
    if constexpr (sizeof(real) == 4) {
        if (d.wide)
            HIPCHK(c, launch_forces_wide(d, r0, count, c->nmax, c->wide_waves,
                                         c->lj_rows * lj_stride_of(c->lj_rows), s));
        else
            HIPCHK(c, launch_forces(d, r0, count, c->tile_waves, s));
    } else {
        HIPCHK(c, launch_forces(d, r0, count, c->tile_waves, s));
    }
    std::vector<double> buf((size_t)count * d.npad * 4);
    HIPCHK(c, hipMemcpyAsync(buf.data(), d.dbg, buf.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int k = 0; k < count; ++k) {
        const double* o = buf.data() + (size_t)k * d.npad * 4;
        if (F)
            for (int a = 0; a < d.n; ++a)
                for (int q = 0; q < 3; ++q)
                    F[((size_t)k * d.n + a) * 3 + q] = o[4 * a + q];
        if (E)
            E[k] = o[3];
    }
    return PAMD_OK;
}

pamd_status pamd_get_forces(pamd_ctx* c, int32_t run, int64_t r0, int32_t count, double* host_F, double* host_E,
                            void* stream)
{
    TraceRange trace_range("pamd_get_forces");
    pamd_status st = check_ctx(c);
    if (st != PAMD_OK)
        return st;
    if (run < 0 || run >= c->n_runs)
        return fail(c, PAMD_ERR_ARG, "run index out of range");
    hipStream_t s = as_stream(stream);
    return c->fp32 ? get_forces_t<float>(c, c->runs[run], r0, count, host_F, host_E, s)
                   : get_forces_t<double>(c, c->runs[run], r0, count, host_F, host_E, s);
}

template <typename real>
static pamd_status get_state_t(pamd_ctx* c, Run& run, double* x, double* v, double* Ep, double* Ek, int32_t* anc,
                               pamd_run_scalars* sc, hipStream_t s)
{
    RunCtl ctl;
    pamd_status st = read_ctl<real>(c, run, &ctl, s);
    if (st != PAMD_OK)
        return st;
    RunDev<real>& d = dev<real>(run);
    const int64_t R = ctl.R_cur;
    const int cur = ctl.cur;
    if (x || v) {
        std::vector<real> buf((size_t)R * 6 * d.npad);
        if (R > 0)
            HIPCHK(c, hipMemcpyAsync(buf.data(), d.slab[cur], buf.size() * sizeof(real), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (int64_t r = 0; r < R; ++r) {
            const real* sl = buf.data() + (size_t)r * 6 * d.npad;
            for (int a = 0; a < d.n; ++a)
                for (int q = 0; q < 3; ++q) {
                    if (x)
                        x[((size_t)r * d.n + a) * 3 + q] = (double)sl[q * d.npad + a];
                    if (v)
                        v[((size_t)r * d.n + a) * 3 + q] = (double)sl[(3 + q) * d.npad + a];
                }
        }
    }
    if (Ep && R > 0)
        HIPCHK(c, hipMemcpyAsync(Ep, d.epot[cur], R * sizeof(double), hipMemcpyDeviceToHost, s));
    if (Ek && R > 0)
        HIPCHK(c, hipMemcpyAsync(Ek, d.ekin[cur], R * sizeof(double), hipMemcpyDeviceToHost, s));
    if (anc && R > 0)
        HIPCHK(c, hipMemcpyAsync(anc, d.anc[cur], R * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (sc) {
        sc->T = ctl.T_cur;
        sc->T_prev = ctl.T_prev;
        sc->sum_lnQ = ctl.sum_lnQ;
        sc->lnQ_last = ctl.lnQ_last;
        sc->R = R;
        sc->step = ctl.step;
        sc->temp_index = ctl.temp_index;
    }
    if (ctl.error)
        return surface_device_error(c, ctl.error);
    return PAMD_OK;
}

pamd_status pamd_get_state(pamd_ctx* c, int32_t run, double* x, double* v, double* E_pot, double* E_kin,
                           int32_t* ancestor, pamd_run_scalars* scalars, void* stream)
{
    TraceRange trace_range("pamd_get_state");
    if (!c)
        return PAMD_ERR_ARG;
    if (run < 0 || run >= c->n_runs)
        return fail(c, PAMD_ERR_ARG, "run index out of range");
    hipStream_t s = as_stream(stream);
    return c->fp32 ? get_state_t<float>(c, c->runs[run], x, v, E_pot, E_kin, ancestor, scalars, s)
                   : get_state_t<double>(c, c->runs[run], x, v, E_pot, E_kin, ancestor, scalars, s);
}

template <typename real>
static pamd_status set_state_t(pamd_ctx* c, Run& run, const double* x, const double* v, const double* Ep,
                               const int32_t* anc, const pamd_run_scalars* sc, hipStream_t s)
{
    RunDev<real>& d = dev<real>(run);
    const int64_t R = sc->R;
    if (R < 1 || R > d.R_cap)
        return fail(c, PAMD_ERR_ARG, "R outside 1..R_cap");
    if (!(sc->T > 0))
        return fail(c, PAMD_ERR_ARG, "T must be > 0");
    RunCtl ctl;
    pamd_status st = read_ctl<real>(c, run, &ctl, s);
    if (st != PAMD_OK)
        return st;
    const int cur = ctl.cur;
    std::vector<real> buf((size_t)R * 6 * d.npad);
    for (int64_t r = 0; r < R; ++r) {
        real* sl = buf.data() + (size_t)r * 6 * d.npad;
        for (int a = 0; a < d.npad; ++a) {
            for (int q = 0; q < 3; ++q) {
                if (a < d.n) {
                    sl[q * d.npad + a] = (real)x[((size_t)r * d.n + a) * 3 + q];
                    sl[(3 + q) * d.npad + a] = (real)v[((size_t)r * d.n + a) * 3 + q];
                } else {
                    sl[q * d.npad + a] = (real)(q == 0 ? 1000 + 10 * a : 1000);
                    sl[(3 + q) * d.npad + a] = (real)0;
                }
            }
        }
    }
    std::vector<double> e(R, 0.0);
    if (Ep)
        e.assign(Ep, Ep + R);
    std::vector<int32_t> an(R);
    for (int64_t r = 0; r < R; ++r)
        an[r] = anc ? anc[r] : (int32_t)r;
    HIPCHK(c, hipMemcpyAsync(d.slab[cur], buf.data(), buf.size() * sizeof(real), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.epot[cur], e.data(), R * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.anc[cur], an.data(), R * sizeof(int32_t), hipMemcpyHostToDevice, s));
    // kinetic energies are evaluated by the next MD call
    HIPCHK(c, hipMemsetAsync(d.ekin[cur], 0, R * sizeof(double), s));
    c->have_energy = Ep ? 1 : 0;   // without energies the next resampling needs an MD call first
    ctl.R_cur = R;
    ctl.R_new = R;
    ctl.T_cur = sc->T;
    ctl.T_prev = sc->T_prev > 0 ? sc->T_prev : sc->T;
    ctl.sum_lnQ = sc->sum_lnQ;
    ctl.lnQ_last = sc->lnQ_last;
    ctl.step = sc->step;
    ctl.temp_index = sc->temp_index;
    ctl.work = 0;
    HIPCHK(c, hipMemcpyAsync(d.ctl, &ctl, sizeof(RunCtl), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return PAMD_OK;
}

pamd_status pamd_set_state(pamd_ctx* c, int32_t run, const double* x, const double* v, const double* E_pot,
                           const int32_t* ancestor, const pamd_run_scalars* scalars, void* stream)
{
    TraceRange trace_range("pamd_set_state");
    pamd_status st = check_ctx(c);
    if (st != PAMD_OK)
        return st;
    if (run < 0 || run >= c->n_runs || !x || !v || !scalars)
        return fail(c, PAMD_ERR_ARG, "bad run index or null state array");
    hipStream_t s = as_stream(stream);
    return c->fp32 ? set_state_t<float>(c, c->runs[run], x, v, E_pot, ancestor, scalars, s)
                   : set_state_t<double>(c, c->runs[run], x, v, E_pot, ancestor, scalars, s);
}

template <typename real>
static pamd_status get_counts_t(pamd_ctx* c, Run& run, int32_t* host_c, int64_t* n, hipStream_t s)
{
    RunCtl ctl;
    pamd_status st = read_ctl<real>(c, run, &ctl, s);
    if (st != PAMD_OK)
        return st;
    const int64_t R = ctl.R_prev;
    if (n)
        *n = R;
    if (host_c && R > 0) {
        HIPCHK(c, hipMemcpyAsync(host_c, dev<real>(run).counts, R * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    return PAMD_OK;
}

pamd_status pamd_get_counts(pamd_ctx* c, int32_t run, int32_t* host_c, int64_t* n, void* stream)
{
    if (!c)
        return PAMD_ERR_ARG;
    if (run < 0 || run >= c->n_runs)
        return fail(c, PAMD_ERR_ARG, "run index out of range");
    hipStream_t s = as_stream(stream);
    return c->fp32 ? get_counts_t<float>(c, c->runs[run], host_c, n, s)
                   : get_counts_t<double>(c, c->runs[run], host_c, n, s);
}

pamd_status pamd_launch_info(const pamd_ctx* c, int32_t* waves_per_block, int32_t* blocks, int32_t* lds_bytes)
{
    if (!c)
        return PAMD_ERR_ARG;
    // the batched launch when there is one, else the register-tile kernel
    if (waves_per_block)
        *waves_per_block = c->wide ? c->wide_waves : c->tile_waves;
    if (blocks)
        *blocks = c->wide ? c->wide_blocks : c->tile_blocks;
    if (lds_bytes)
        *lds_bytes = (int32_t)(c->wide ? c->wide_lds : c->tile_lds);
    return PAMD_OK;
}

pamd_status pamd_run_launch(const pamd_ctx* c, int32_t run, int32_t* layout, int32_t* waves_per_block,
                            int32_t* blocks, int32_t* lds_bytes)
{
    if (!c || run < 0 || run >= c->n_runs)
        return PAMD_ERR_ARG;
    const int w = c->fp32 && c->runs[run].f.wide;
    if (layout)
        *layout = w ? PAMD_LAYOUT_WIDE : PAMD_LAYOUT_TILE;
    if (waves_per_block)
        *waves_per_block = w ? c->wide_waves : c->tile_waves;
    if (blocks)
        *blocks = w ? c->wide_blocks
                    : tile_launch_blocks(c, c->fp32 ? c->runs[run].f.R_cap : c->runs[run].d.R_cap);
    if (lds_bytes)
        *lds_bytes = (int32_t)(w ? c->wide_lds : c->tile_lds);
    return PAMD_OK;
}

pamd_status pamd_set_schedule(pamd_ctx* c, int32_t run, const double* T, int32_t n, void* stream)
{
    TraceRange trace_range("pamd_set_schedule");
    pamd_status st = check_ctx(c);
    if (st != PAMD_OK)
        return st;
    if (run < 0 || run >= c->n_runs || !T || n < 1 || n > kMaxSched)
        return fail(c, PAMD_ERR_ARG, "bad run index or schedule length (1.." + std::to_string(kMaxSched) + ")");
    for (int i = 0; i < n; ++i)
        if (!(T[i] > 0.0))
            return fail(c, PAMD_ERR_ARG, "schedule temperatures must be > 0");
    hipStream_t s = as_stream(stream);
    Run& r = c->runs[run];
    const double* dst = c->fp32 ? r.f.sched : r.d.sched;
    HIPCHK(c, hipMemcpyAsync((void*)dst, T, sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    r.f.n_sched = n;
    r.d.n_sched = n;
    return PAMD_OK;
}

static void drop_graph(pamd_ctx* c, int slot)
{
    if (c->graph_exec[slot])
        (void)hipGraphExecDestroy(c->graph_exec[slot]);
    if (c->graph[slot])
        (void)hipGraphDestroy(c->graph[slot]);
    c->graph_exec[slot] = nullptr;
    c->graph[slot] = nullptr;
}

pamd_status pamd_graph_capture(pamd_ctx* c, int32_t slot, int32_t parts, int32_t n_steps, int32_t mode,
                               void* stream)
{
    TraceRange trace_range("pamd_graph_capture");
    pamd_status st = check_ctx(c);
    if (st != PAMD_OK)
        return st;
    if (!stream)
        return fail(c, PAMD_ERR_ARG, "graph capture needs a non-null stream");
    if (slot < 0 || slot >= kGraphSlots || parts < 1 || parts > 3 || n_steps < 0 || (mode != 0 && mode != 1))
        return fail(c, PAMD_ERR_ARG, "bad graph slot, parts, n_steps or schedule mode");
    hipStream_t s = as_stream(stream);
    drop_graph(c, slot);
    HIPCHK(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    std::vector<double> req(c->n_runs, mode == 0 ? 0.0 : -1.0);
    pamd_status b = PAMD_OK;
    if (parts & 1)
        b = pamd_resample(c, req.data(), nullptr, stream);
    if (b == PAMD_OK && (parts & 2))
        b = pamd_md_steps(c, n_steps, stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (b != PAMD_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return b;
    }
    if (e != hipSuccess)
        return fail(c, PAMD_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    c->graph[slot] = g;
    HIPCHK(c, hipGraphInstantiate(&c->graph_exec[slot], g, nullptr, nullptr, 0));
    return PAMD_OK;
}

pamd_status pamd_graph_launch(pamd_ctx* c, int32_t slot, void* stream)
{
    TraceRange trace_range("pamd_graph_launch");
    pamd_status st = check_ctx(c);
    if (st != PAMD_OK)
        return st;
    if (slot < 0 || slot >= kGraphSlots || !c->graph_exec[slot])
        return fail(c, PAMD_ERR_STATE, "no captured graph in this slot");
    HIPCHK(c, hipGraphLaunch(c->graph_exec[slot], as_stream(stream)));
    return PAMD_OK;
}

pamd_status pamd_export_configs(pamd_ctx* c, int32_t run, int64_t r0, int64_t count, float* d_x, float* d_F_nb,
                                void* stream)
{
    TraceRange trace_range("pamd_export_configs");
    pamd_status st = check_ctx(c);
    if (st != PAMD_OK)
        return st;
    if (run < 0 || run >= c->n_runs)
        return fail(c, PAMD_ERR_ARG, "run index out of range");
    if (!c->fp32 || c->runs[run].f.wide)
        return fail(c, PAMD_ERR_ARG, "configuration export needs an FP32 run in the register-tile layout (up to " +
                                         std::to_string(PAMD_TILE_ATOMS) + " atoms)");
    const RunDev<float>& d = c->runs[run].f;
    if (r0 < 0 || count < 0 || r0 + count > d.R_cap || (count > 0 && (!d_x || !d_F_nb)))
        return fail(c, PAMD_ERR_ARG, "replica range or output arrays invalid");
    if (count == 0)
        return PAMD_OK;
    HIPCHK(c, launch_export(d, r0, count, d_x, d_F_nb, c->tile_waves, as_stream(stream)));
    return PAMD_OK;
}

// r-RESPA buffers of every run, carved in run order
static size_t carve_mts_all(pamd_ctx* c, void* base)
{
    nn::SpanCarver cv(base);
    for (auto& run : c->runs) {
        const RunDev<float>& d = run.f;
        const nn::MtsBuffers b = nn::carve_mts(cv, d.R_cap, d.n, d.npad);
        if (base)
            run.mts = b;
    }
    return cv.off;
}

pamd_status pamd_mts_query_sizes(pamd_ctx* c, size_t* bytes)
{
    pamd_status st = check_ctx(c);
    if (st != PAMD_OK)
        return st;
    if (!bytes)
        return fail(c, PAMD_ERR_ARG, "null output");
    *bytes = carve_mts_all(c, nullptr);
    return PAMD_OK;
}

pamd_status pamd_set_mts(pamd_ctx* c, pamd_nn* nn, int32_t outer_ratio, void* d_mem, size_t mem_bytes,
                         void* stream)
{
    pamd_status st = check_ctx(c);
    if (st != PAMD_OK)
        return st;
    hipStream_t s = as_stream(stream);
    HIPCHK(c, hipStreamSynchronize(s));
    if (!nn) {
        for (auto& run : c->runs)
            run.mts = nn::MtsBuffers{};
        c->nn = nullptr;
        c->mts_ratio = 0;
        return PAMD_OK;
    }
    if (!c->fp32 || c->wide)
        return fail(c, PAMD_ERR_ARG, "r-RESPA with the surrogate needs an FP32 context whose runs all use the "
                                     "register-tile layout (molecules up to " + std::to_string(PAMD_TILE_ATOMS) +
                                     " atoms)");
    if (outer_ratio < 1)
        return fail(c, PAMD_ERR_ARG, "outer_ratio must be >= 1");
    if (c->runs[0].f.thermostat != PAMD_THERMOSTAT_ANDERSEN)
        return fail(c, PAMD_ERR_ARG, "r-RESPA with the surrogate runs with the Andersen bath only");
    for (auto& run : c->runs)
        if (run.f.n != nn->topo.n)
            return fail(c, PAMD_ERR_ARG, "surrogate atom count differs from a run's");
    if (!d_mem || (reinterpret_cast<uintptr_t>(d_mem) & (kAlign - 1)) != 0)
        return fail(c, PAMD_ERR_ARG, "r-RESPA buffer missing or not 256-byte aligned");
    if (mem_bytes < carve_mts_all(c, nullptr))
        return fail(c, PAMD_ERR_ARG, "r-RESPA buffer smaller than pamd_mts_query_sizes");
    carve_mts_all(c, d_mem);
    c->nn = nn;
    c->mts_ratio = outer_ratio;
    return PAMD_OK;
}

void pamd_destroy(pamd_ctx* c)
{
    if (!c)
        return;
    for (int g = 0; g < kGraphSlots; ++g)
        drop_graph(c, g);
    for (int k = 0; k < pamd_ctx::kSide; ++k) {
        if (c->side[k])
            (void)hipStreamSynchronize(c->side[k]);
        if (c->side[k])
            (void)hipStreamDestroy(c->side[k]);
        if (c->ev_join[k])
            (void)hipEventDestroy(c->ev_join[k]);
    }
    if (c->ev_fork)
        (void)hipEventDestroy(c->ev_fork);
    delete c;
}

const char* pamd_last_error(const pamd_ctx* c)
{
    if (!c)
        return "null context";
    return c->err.c_str();
}

