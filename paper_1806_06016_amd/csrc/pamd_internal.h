// Internal structures shared by the HIP kernels and the host runtime of libpamd.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pamd.h"

namespace pamd {

constexpr int kRow = 16;            // lanes per replica (one DPP row)
constexpr int kRowsPerWave = 4;     // replicas per wave64
constexpr int kMaxSlots = 5;        // 16-atom blocks held in registers (N <= 80)
constexpr int kWaveSize = 64;
constexpr int kMaxSched = 4096;  // temperatures a device schedule can hold
// wide layout (molecules of up to 320 atoms, and every run of a context that
// holds one): one replica per wavefront, atom a on lane a % 64, slot a / 64
constexpr int kWide = 64;
constexpr int kWideSlots = 5;
constexpr int kWideMaxAtoms = kWide * kWideSlots;
// parameters per angle group: six angle pairs (k, theta0), four bonds (k_b, r0)
constexpr int kAngPar = 20;
// LJ class table of the wide layout: the pair coefficients of every pair of
// distinct per-atom (sigma, epsilon) values (a molecule in the wide layout has
// at most PAMD_WIDE_LJ_CLASSES of them).  A context sizes its tables to its
// largest class count m: m + 1 rows (the last one all zero, for padding
// atoms), an odd row stride so consecutive rows start in different banks;
// every run's device table has room for the largest shape.
constexpr int kLjClasses = PAMD_WIDE_LJ_CLASSES + 1;
constexpr int kLjStride = kLjClasses + 1;
__host__ __device__ constexpr int lj_stride_of(int rows) { return rows | 1; }

// Number of tile steps of the all-pairs schedule for `nslot` blocks of 16 atoms:
// each diagonal block takes 8 row rotations (k = 1..8, k = 8 half-masked),
// each off-diagonal block pair takes 16 (k = 0..15).
__host__ __device__ constexpr int tile_steps(int nslot) { return nslot * 8 + nslot * (nslot - 1) / 2 * 16; }

// Device-resident control block of one run.  Everything that changes from
// one temperature to the next lives here, so the per-temperature kernel
// sequence needs no host values and can be replayed from a HIP graph.
struct alignas(64) RunCtl {
    double T_cur;        // bath temperature of the current population
    double T_prev;
    double T_next;       // chosen by the weights kernel (requested or adaptive)
    double T_req;        // last request: > 0 explicit T, 0 adaptive, < 0 device schedule
    double dbeta;        // 1/(kB T_next) - 1/(kB T_cur)
    double m;            // min E
    double S;            // sum exp(-dbeta (E - m))
    double S2;           // sum exp(-2 dbeta (E - m))
    double lnQ_last;
    double sum_lnQ;
    double V_last;
    int64_t R_cur;       // current population size
    int64_t R_new;       // size after the pending resampling
    int64_t R_prev;      // size before the last resampling (length of the counts array)
    uint32_t step;       // global MD step counter (Philox counter word 1)
    uint32_t temp_index; // i
    int32_t cur;         // ping-pong buffer holding the current population
    int32_t error;       // sticky PAMD_ERR_* code
    int32_t work;        // persistent-kernel work counter
    int32_t frozen;      // error != 0 when the current MD call began: its kernels leave the run unchanged
    uint32_t ticket;     // blocks done in the current multi-block reduction (the last one finishes it)
    int32_t w_phase;     // adaptive step: 0 probe at the largest step, 1 Newton iterations, 2 T_next fixed
    int32_t w_iter;      // Newton iterations done
    int32_t pad;
    double w_b, w_lo, w_hi;   // adaptive step: current dbeta and its bracket
    double w_var;        // population variance of E (start of the Newton iteration)
};

// operations of one r-RESPA kernel pass (k_respa), applied in this order
enum : int { kRespaInnerKick = 1, kRespaOuterEnd = 2, kRespaCollide = 4, kRespaOuterStart = 8, kRespaDrift = 16 };

// Per-run device pointers and constants (passed by value to kernels).
template <typename real>
struct RunDev {
    RunCtl* ctl;
    real* slab[2];          // [R_cap][6][npad]  x | y | z | vx | vy | vz
    double* epot[2];        // [R_cap]
    double* ekin[2];        // [R_cap] (ping-pong with the slabs)
    int32_t* anc[2];        // [R_cap]
    int32_t* counts;        // [R_cap]
    int32_t* src_of;        // [R_cap]
    double* cdf;            // [R_cap] running weight sums W_j (multinomial resampling)
    double* part;           // per-block partial sums of the multi-block reductions
    int64_t* cpart;         // per-block copy-number sums / family counts [ceil(R_cap / 256)]
    uint8_t* fam;           // [R_target] family flags
    const double* unif;     // optional caller uniforms for this run
    // topology / parameters
    const real* nb_ab;      // [steps][16][2]   (12 c12 s, -6 c6 s)
    const real* nb_c;       // [steps][16]      Coulomb coefficient
    const int4* bidx;       // [nb]   (i, j, -, -) of the bonds no angle group evaluates
    const real* bpar;       // [nb][2] (k, r0)
    const int4* agrp;       // [nag][2] angle groups: (j, o0, o1, o2), (o3, -, -, -), -1 = none;
                            // slots [0, nag6) hold four outer atoms, the rest at most three (o0..o2)
    const real* agpar;      // [nag][kAngPar]: (k, theta0) of the outer pairs (0,1) (0,2) (0,3) (1,2)
                            // (1,3) (2,3), then (k_b, r0) of the bond centre - outer atom a, a = 0..3
                            // (k_b = 0 where the bond is another group's or a bond pass's)
    const int4* dgrp;       // [ng][2] dihedral groups: (j, k, i0, i1), (i2, l0, l1, l2), -1 = none
    const real* dgpar;      // [ng][9][5] (k cos(delta), n, c0, c1, c2) of (i_a, l_c) at 3 a + c, with
                            // k cos(delta) n U_{n-1}(c) = c0 + c1 c + c2 c^2 when n <= 3
    const double* mass;     // [npad] (0 for padding)
    const double* x_init;   // [n][3]
    const double* sched;    // device temperature schedule [kMaxSched]
    int32_t n_sched;        // its length (set by pamd_set_schedule; 0 = none)
    double* dbg;            // force-debug scratch [PAMD_FORCE_CHUNK][npad][4]
    void* obs;              // device pamd_obs
    int32_t n, npad, nslot, nb, nag, ng;
    int32_t nag6;           // angle slots of the six-angle body
    int32_t dih_general;    // some torsion has n > 3: its derivative by the Chebyshev recurrence
    int64_t R_target, R_cap;
    double kB, dt, T0, V_target, T_final;
    uint32_t p24;           // Andersen threshold: collide iff (w >> 8) < p24
    uint32_t key0, key1;    // Philox key
    int32_t dielectric;
    int32_t waves_per_block;
    int32_t resampling;     // PAMD_RESAMPLE_*
    int32_t thermostat;     // PAMD_THERMOSTAT_*
    double lc1, lc2;        // Langevin: exp(-gamma dt), sqrt(1 - exp(-2 gamma dt))
    // wide layout only: per-atom (q sqrt(k_e c), LJ class) with c = 1/2 for
    // eps = 4r and 1 in vacuum, the LJ class table, and per (atom, 32-atom
    // chunk) the bit masks (excluded pair incl. self, scaled 1-4 pair)
    const float2* apar2;    // [n]
    const float2* ljtab;    // [lj_pad + 1][lj_stride] (12 c12, -6 c6) of class pairs (a, b)
    int32_t lj_stride;      // row stride of the class table (float2)
    int32_t lj_pad;         // the all-zero class of padding atoms (last row)
    const uint2* pmask;     // [n][nchunk]
    const uint64_t* stepmask;   // [t][s] (5 x 5): bit k set when some lane of own slot s meets an
                                // excluded or 1-4 partner of slot t at rotation step k
    int32_t nchunk;
    int32_t wide;
    float s14lj, s14c;
};

}  // namespace pamd
