// Internal definitions shared by the host loader, the kernels and the C-ABI
// entry points of the gfx950 kinetics library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/ck.h"

namespace ck {

constexpr int kWave = 64;
constexpr int kMaxSlots = 6;      // reactant + product species slots per reaction (3 + 3)
constexpr int kMaxN = 128;        // largest state size (T + 127 species)

// Reaction classes; the loader orders reactions by class so lanes of one
// wavefront mostly take the same branch.
enum RxnType { kElementary = 0, kThirdBody = 1, kLindemann = 2, kTroe = 3 };

// One reaction, packed into 64 bytes so a lane fetches it with four 16-byte loads.
// Reactions are stored sorted by type so lanes of one wavefront mostly share a branch.
struct RxnRec {
    double lnA, beta, EaR;      // ln A, temperature exponent, E/R (high-pressure limit for fall-off)
    double dnu;                 // net mole change sum_j (nu''_j - nu'_j)
    int meta;                   // bits 0-1 type, bit 2 reversible, bits 3-5 slots, bits 6-8 reactant slots,
                                // bits 9-31 number of third-body efficiencies
    int eff_begin;              // first entry in the efficiency table
    int sp[3];                  // species of slots 0..5, two 16-bit indices per int (reactants first)
    int nu;                     // stoichiometric coefficient of slot s in bits 2s..2s+1 (1..3)
    int fall;                   // index into the fall-off table, or -1
    int blk_slots;              // largest slot count among the 64 stored reactions of this one's block
};

struct FallRec {                // fall-off parameters (Lindemann / Troe)
    double lnA0, beta0, Ea0R;   // low-pressure limit
    double a, invT3, invT1, T2; // Troe centring parameters (1/T*** and 1/T* stored)
    double pad;
};

struct EffRec {                 // third-body efficiency alpha of one species, stored as alpha - 1
    double am1;
    int sp, pad;
};

__host__ __device__ inline int rx_type(int meta) { return meta & 3; }
__host__ __device__ inline int rx_rev(int meta) { return (meta >> 2) & 1; }
__host__ __device__ inline int rx_nslot(int meta) { return (meta >> 3) & 7; }
__host__ __device__ inline int rx_nreac(int meta) { return (meta >> 6) & 7; }
__host__ __device__ inline int rx_neff(int meta) { return meta >> 9; }
__host__ __device__ inline int rx_sp(const RxnRec &r, int s) { return (r.sp[s >> 1] >> (16 * (s & 1))) & 0xffff; }
__host__ __device__ inline int rx_nu(const RxnRec &r, int s) { return (r.nu >> (2 * s)) & 3; }

// Device view of a mechanism.
struct DevMech {
    int nsp, nrxn, N, n_eff;
    double R;            // J/(mol K)
    double ln_p0_R;      // ln(p0 / R), so ln(p0/(R T)) = ln_p0_R - ln T
    // species block, [3 + kThermoCoef][nsp]: W, 1/W, Tmid, then the NASA-7 derived coefficients;
    // per range r (0 low, 1 high) at thermo offset 21*r:
    //   cp/R   : c0..c4           (a1, a2, a3, a4, a5)
    //   H/(RT) : c5..c10          (a1, a2/2, a3/3, a4/4, a5/5, a6)
    //   S/R    : c11..c16         (a1 [ln T], a2, a3/2, a4/3, a5/4, a7)
    //   dcp/dT : c17..c20         (a2, 2 a3, 3 a4, 4 a5)
    const double *spd;
    const RxnRec *rx;
    const FallRec *fall;
    const EffRec *eff;
    const int *orig_index;       // file order of each stored reaction
    __host__ __device__ const double *W() const { return spd; }
    __host__ __device__ const double *invW() const { return spd + nsp; }
    __host__ __device__ const double *Tmid() const { return spd + 2 * nsp; }
    __host__ __device__ const double *thermo() const { return spd + 3 * nsp; }
};

constexpr int kThermoCoef = 42;

struct HostMech {
    int nsp = 0, nrxn = 0, nel = 0;
    double R = 0, p0 = 0;
    std::vector<double> W, Tmid, alow, ahigh;    // alow/ahigh: 7 per species
    struct Rxn {
        int type = 0, rev = 1;
        std::vector<int> rsp, rnu, psp, pnu;
        double A = 0, beta = 0, Ea = 0;
        double A0 = 0, beta0 = 0, Ea0 = 0;
        double ta = 0, T3 = 0, T1 = 0, T2 = 0;
        std::vector<std::pair<int, double>> eff;
    };
    std::vector<Rxn> rx;
};

int parse_mechanism(const char *path, HostMech &hm);

}  // namespace ck

struct ck_mech {
    int device = 0;
    ck::HostMech host;
    ck::DevMech dev{};
    void *dev_block = nullptr;      // single device allocation holding every table
    size_t dev_bytes = 0;
    // Library-owned workspaces for calls that pass workspace == NULL: one per stream, so
    // calls on different streams never share a queue counter or parking area (calls on one
    // stream are ordered by the stream).  Guarded by ws_mutex; freed by ck_mechanism_free.
    struct StreamWs {
        hipStream_t stream;
        void *ptr;
        size_t bytes;
    };
    std::mutex ws_mutex;
    std::vector<StreamWs> ws;
};

#define CK_HIP_TRY(expr)                       \
    do {                                       \
        hipError_t _e = (expr);                \
        if (_e != hipSuccess) return CK_EHIP;  \
    } while (0)
