// Internal definitions shared by the host loader, the kernels and the C-ABI
// entry points of the gfx950 kinetics library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/ck.h"

namespace ck {

constexpr int kWave = 64;
constexpr int kMaxSlots = 6;      // reactant + product species slots per reaction (3 + 3)
constexpr int kMaxN = 128;        // largest state size (T + 127 species)

// Reaction classes; the loader orders reactions by class so lanes of one
// wavefront mostly take the same branch.
enum RxnType { kElementary = 0, kThirdBody = 1, kLindemann = 2, kTroe = 3 };

// Device view of a mechanism: structure-of-arrays over species and reactions.
struct DevMech {
    int nsp, nrxn, N;
    int n_eff;
    double R;            // J/(mol K)
    double ln_p0_R;      // ln(p0 / R), so ln(p0/(R T)) = ln_p0_R - ln T

    // species [nsp]
    const double *W, *invW, *Tmid;
    // NASA-7 derived coefficients, [kThermoCoef][nsp]; per range r (0 low, 1 high) at offset 21*r:
    //   cp/R   : c0..c4           (a1, a2, a3, a4, a5)
    //   H/(RT) : c5..c10          (a1, a2/2, a3/3, a4/4, a5/5, a6)
    //   S/R    : c11..c16         (a1 [ln T], a2, a3/2, a4/3, a5/4, a7)
    //   dcp/dT : c17..c20         (a2, 2 a3, 3 a4, 4 a5)
    const double *thermo;

    // reactions [nrxn], sorted by type
    const double *lnA, *beta, *EaR, *dnu;
    const int *type, *rev, *nslot, *nreac;      // nslot = reactant + product slots; nreac = reactant slots
    const int *slot_sp;                          // [kMaxSlots][nrxn]
    const int *slot_nu;                          // [kMaxSlots][nrxn], stoichiometric coefficient (> 0)
    const int *eff_begin, *eff_count;            // into eff_sp / eff_am1
    const int *eff_sp;
    const double *eff_am1;                       // alpha - 1
    const double *lnA0, *beta0, *Ea0R;           // fall-off low-pressure limit
    const double *troe_a, *troe_invT3, *troe_invT1, *troe_T2;
    const int *orig_index;                       // file order of each sorted reaction
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
    // workspace cache for calls that pass workspace == NULL
    void *ws = nullptr;
    size_t ws_bytes = 0;
};

#define CK_HIP_TRY(expr)                       \
    do {                                       \
        hipError_t _e = (expr);                \
        if (_e != hipSuccess) return CK_EHIP;  \
    } while (0)
