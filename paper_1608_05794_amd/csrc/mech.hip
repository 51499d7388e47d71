// Mechanism staging: parse the CKMECH text format, pack structure-of-arrays
// tables and upload them in one device allocation (Section 3 data: NASA-7
// thermodynamics per species, modified Arrhenius rates, stoichiometry,
// third-body efficiencies and fall-off parameters per reaction).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <numeric>
#include <sstream>
#include <string>

#include "ck_internal.h"

namespace ck {

namespace {

struct Reader {
    std::ifstream in;
    bool ok = true;
    template <class T>
    T get() {
        T v{};
        if (!(in >> v)) ok = false;
        return v;
    }
    bool word(const char *w) {
        std::string s;
        if (!(in >> s) || s != w) ok = false;
        return ok;
    }
};

}  // namespace

int parse_mechanism(const char *path, HostMech &hm) {
    Reader r;
    r.in.open(path);
    if (!r.in) return CK_EIO;
    if (!r.word("CKMECH") || r.get<int>() != 1 || !r.ok) return CK_EPARSE;
    if (!r.word("CONST")) return CK_EPARSE;
    hm.R = r.get<double>();
    hm.p0 = r.get<double>();
    if (!r.word("ELEMENTS")) return CK_EPARSE;
    hm.nel = r.get<int>();
    if (!r.ok || hm.nel < 1 || hm.nel > 64) return CK_EPARSE;
    for (int e = 0; e < hm.nel; e++) {
        r.word("E");
        r.get<std::string>();
        r.get<double>();
    }
    if (!r.word("SPECIES")) return CK_EPARSE;
    hm.nsp = r.get<int>();
    if (!r.ok || hm.nsp < 1 || hm.nsp + 1 > kMaxN) return r.ok ? CK_EUNSUPPORTED : CK_EPARSE;
    hm.W.resize(hm.nsp);
    hm.Tmid.resize(hm.nsp);
    hm.alow.resize(7 * hm.nsp);
    hm.ahigh.resize(7 * hm.nsp);
    for (int k = 0; k < hm.nsp; k++) {
        r.word("S");
        r.get<std::string>();
        hm.W[k] = r.get<double>();
        int nc = r.get<int>();
        if (!r.ok || nc < 0 || nc > hm.nel) return CK_EPARSE;
        for (int c = 0; c < nc; c++) {
            int e = r.get<int>();
            r.get<int>();
            if (e < 0 || e >= hm.nel) return CK_EPARSE;
        }
        r.get<double>();
        hm.Tmid[k] = r.get<double>();
        r.get<double>();
        for (int j = 0; j < 7; j++) hm.alow[7 * k + j] = r.get<double>();
        for (int j = 0; j < 7; j++) hm.ahigh[7 * k + j] = r.get<double>();
        if (!r.ok || !(hm.W[k] > 0)) return CK_EPARSE;
    }
    if (!r.word("REACTIONS")) return CK_EPARSE;
    hm.nrxn = r.get<int>();
    if (!r.ok || hm.nrxn < 0) return CK_EPARSE;
    hm.rx.resize(hm.nrxn);
    for (auto &x : hm.rx) {
        if (!r.word("R")) return CK_EPARSE;
        x.type = r.get<int>();
        x.rev = r.get<int>();
        int nr = r.get<int>();
        if (!r.ok || x.type < 0 || x.type > 3 || nr < 1 || nr > 3) return CK_EPARSE;
        for (int j = 0; j < nr; j++) {
            x.rsp.push_back(r.get<int>());
            x.rnu.push_back(r.get<int>());
        }
        int np = r.get<int>();
        if (!r.ok || np < 1 || np > 3) return CK_EPARSE;
        for (int j = 0; j < np; j++) {
            x.psp.push_back(r.get<int>());
            x.pnu.push_back(r.get<int>());
        }
        for (int j = 0; j < nr; j++)
            if (x.rsp[j] < 0 || x.rsp[j] >= hm.nsp || x.rnu[j] < 1 || x.rnu[j] > 3) return CK_EPARSE;
        for (int j = 0; j < np; j++)
            if (x.psp[j] < 0 || x.psp[j] >= hm.nsp || x.pnu[j] < 1 || x.pnu[j] > 3) return CK_EPARSE;
        x.A = r.get<double>();
        x.beta = r.get<double>();
        x.Ea = r.get<double>();
        if (x.type >= 2) {
            x.A0 = r.get<double>();
            x.beta0 = r.get<double>();
            x.Ea0 = r.get<double>();
        }
        if (x.type == 3) {
            x.ta = r.get<double>();
            x.T3 = r.get<double>();
            x.T1 = r.get<double>();
            x.T2 = r.get<double>();
        }
        if (x.type >= 1) {
            int ne = r.get<int>();
            if (!r.ok || ne < 0 || ne > hm.nsp) return CK_EPARSE;
            for (int j = 0; j < ne; j++) {
                int s = r.get<int>();
                double a = r.get<double>();
                if (s < 0 || s >= hm.nsp) return CK_EPARSE;
                x.eff.emplace_back(s, a);
            }
        }
        if (!r.ok || !(x.A > 0) || (x.type >= 2 && !(x.A0 > 0))) return CK_EPARSE;
    }
    if (!r.word("END")) return CK_EPARSE;
    return CK_OK;
}

}  // namespace ck

using namespace ck;

namespace {

// Byte layout of the single device block: each table starts 256-byte aligned.
struct Packer {
    std::vector<char> buf;
    size_t add(const void *src, size_t bytes) {
        size_t off = (buf.size() + 255) & ~size_t(255);
        buf.resize(off + std::max<size_t>(bytes, 8));
        if (bytes) std::memcpy(buf.data() + off, src, bytes);
        return off;
    }
    template <class T>
    size_t add(const std::vector<T> &v) { return add(v.data(), v.size() * sizeof(T)); }
};

}  // namespace

extern "C" int ck_mechanism_load(const char *path, int device, ck_mech **out) {
    if (!path || !out) return CK_EINVAL;
    *out = nullptr;
    auto *m = new (std::nothrow) ck_mech;
    if (!m) return CK_ENOMEM;
    int rc = parse_mechanism(path, m->host);
    if (rc != CK_OK) {
        delete m;
        return rc;
    }
    const HostMech &hm = m->host;
    const int ns = hm.nsp, nr = hm.nrxn;

    // species tables
    std::vector<double> W(ns), invW(ns), Tmid(ns), th(size_t(kThermoCoef) * ns);
    for (int k = 0; k < ns; k++) {
        W[k] = hm.W[k];
        invW[k] = 1.0 / hm.W[k];
        Tmid[k] = hm.Tmid[k];
        for (int rg = 0; rg < 2; rg++) {
            const double *a = rg == 0 ? &hm.alow[7 * k] : &hm.ahigh[7 * k];
            double c[21] = {a[0], a[1], a[2], a[3], a[4],
                            a[0], a[1] / 2.0, a[2] / 3.0, a[3] / 4.0, a[4] / 5.0, a[5],
                            a[0], a[1], a[2] / 2.0, a[3] / 3.0, a[4] / 4.0, a[6],
                            a[1], 2.0 * a[2], 3.0 * a[3], 4.0 * a[4]};
            for (int j = 0; j < 21; j++) th[size_t(21 * rg + j) * ns + k] = c[j];
        }
    }
    // reactions sorted by type (stable), so wavefront lanes mostly share a branch
    std::vector<int> order(nr);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hm.rx[a].type < hm.rx[b].type; });
    std::vector<double> lnA(nr), beta(nr), EaR(nr), dnu(nr), lnA0(nr), beta0(nr), Ea0R(nr);
    std::vector<double> ta(nr), iT3(nr), iT1(nr), T2(nr);
    std::vector<int> type(nr), rev(nr), nslot(nr), nreac(nr), sp(size_t(kMaxSlots) * std::max(nr, 1), 0),
        nu(size_t(kMaxSlots) * std::max(nr, 1), 0), eb(nr), ec(nr), orig(nr), esp;
    std::vector<double> eam1;
    for (int ii = 0; ii < nr; ii++) {
        const auto &x = hm.rx[order[ii]];
        orig[ii] = order[ii];
        lnA[ii] = std::log(x.A);
        beta[ii] = x.beta;
        EaR[ii] = x.Ea / hm.R;
        type[ii] = x.type;
        rev[ii] = x.rev;
        int s = 0;
        double d = 0;
        for (size_t j = 0; j < x.rsp.size(); j++, s++) {
            sp[size_t(s) * nr + ii] = x.rsp[j];
            nu[size_t(s) * nr + ii] = x.rnu[j];
            d -= x.rnu[j];
        }
        nreac[ii] = s;
        for (size_t j = 0; j < x.psp.size(); j++, s++) {
            sp[size_t(s) * nr + ii] = x.psp[j];
            nu[size_t(s) * nr + ii] = x.pnu[j];
            d += x.pnu[j];
        }
        nslot[ii] = s;
        dnu[ii] = d;
        lnA0[ii] = x.type >= 2 ? std::log(x.A0) : 0.0;
        beta0[ii] = x.beta0;
        Ea0R[ii] = x.Ea0 / hm.R;
        ta[ii] = x.ta;
        iT3[ii] = x.type == 3 ? 1.0 / x.T3 : 0.0;
        iT1[ii] = x.type == 3 ? 1.0 / x.T1 : 0.0;
        T2[ii] = x.T2;
        eb[ii] = int(esp.size());
        for (auto &e : x.eff) {
            esp.push_back(e.first);
            eam1.push_back(e.second - 1.0);
        }
        ec[ii] = int(esp.size()) - eb[ii];
    }

    Packer pk;
    size_t oW = pk.add(W), oiW = pk.add(invW), oT = pk.add(Tmid), oth = pk.add(th);
    size_t olnA = pk.add(lnA), obeta = pk.add(beta), oEaR = pk.add(EaR), odnu = pk.add(dnu);
    size_t otype = pk.add(type), orev = pk.add(rev), onslot = pk.add(nslot), onreac = pk.add(nreac);
    size_t osp = pk.add(sp), onu = pk.add(nu), oeb = pk.add(eb), oec = pk.add(ec), oesp = pk.add(esp),
           oeam1 = pk.add(eam1);
    size_t olnA0 = pk.add(lnA0), obeta0 = pk.add(beta0), oEa0R = pk.add(Ea0R);
    size_t ota = pk.add(ta), oiT3 = pk.add(iT3), oiT1 = pk.add(iT1), oT2 = pk.add(T2), oorig = pk.add(orig);

    m->device = device;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) {
        delete m;
        return CK_EHIP;
    }
    if (hipSetDevice(device) != hipSuccess) {
        delete m;
        return CK_EINVAL;
    }
    void *blk = nullptr;
    if (hipMalloc(&blk, pk.buf.size()) != hipSuccess) {
        hipSetDevice(prev);
        delete m;
        return CK_ENOMEM;
    }
    if (hipMemcpy(blk, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(blk);
        hipSetDevice(prev);
        delete m;
        return CK_EHIP;
    }
    hipSetDevice(prev);
    m->dev_block = blk;
    m->dev_bytes = pk.buf.size();
    char *b = static_cast<char *>(blk);
    DevMech &d = m->dev;
    d.nsp = ns;
    d.nrxn = nr;
    d.N = ns + 1;
    d.n_eff = int(esp.size());
    d.R = hm.R;
    d.ln_p0_R = std::log(hm.p0 / hm.R);
    d.W = reinterpret_cast<const double *>(b + oW);
    d.invW = reinterpret_cast<const double *>(b + oiW);
    d.Tmid = reinterpret_cast<const double *>(b + oT);
    d.thermo = reinterpret_cast<const double *>(b + oth);
    d.lnA = reinterpret_cast<const double *>(b + olnA);
    d.beta = reinterpret_cast<const double *>(b + obeta);
    d.EaR = reinterpret_cast<const double *>(b + oEaR);
    d.dnu = reinterpret_cast<const double *>(b + odnu);
    d.type = reinterpret_cast<const int *>(b + otype);
    d.rev = reinterpret_cast<const int *>(b + orev);
    d.nslot = reinterpret_cast<const int *>(b + onslot);
    d.nreac = reinterpret_cast<const int *>(b + onreac);
    d.slot_sp = reinterpret_cast<const int *>(b + osp);
    d.slot_nu = reinterpret_cast<const int *>(b + onu);
    d.eff_begin = reinterpret_cast<const int *>(b + oeb);
    d.eff_count = reinterpret_cast<const int *>(b + oec);
    d.eff_sp = reinterpret_cast<const int *>(b + oesp);
    d.eff_am1 = reinterpret_cast<const double *>(b + oeam1);
    d.lnA0 = reinterpret_cast<const double *>(b + olnA0);
    d.beta0 = reinterpret_cast<const double *>(b + obeta0);
    d.Ea0R = reinterpret_cast<const double *>(b + oEa0R);
    d.troe_a = reinterpret_cast<const double *>(b + ota);
    d.troe_invT3 = reinterpret_cast<const double *>(b + oiT3);
    d.troe_invT1 = reinterpret_cast<const double *>(b + oiT1);
    d.troe_T2 = reinterpret_cast<const double *>(b + oT2);
    d.orig_index = reinterpret_cast<const int *>(b + oorig);
    *out = m;
    return CK_OK;
}

extern "C" void ck_mechanism_free(ck_mech *m) {
    if (!m) return;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(m->device);
    if (m->dev_block) hipFree(m->dev_block);
    if (m->ws) hipFree(m->ws);
    hipSetDevice(prev);
    delete m;
}

extern "C" int ck_mechanism_info(const ck_mech *m, int *n_species, int *n_reactions, int *n_elements) {
    if (!m) return CK_EINVAL;
    if (n_species) *n_species = m->host.nsp;
    if (n_reactions) *n_reactions = m->host.nrxn;
    if (n_elements) *n_elements = m->host.nel;
    return CK_OK;
}
