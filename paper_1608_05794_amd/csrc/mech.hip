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

    // species block: W, 1/W, Tmid, then the derived NASA-7 coefficients, each [nsp]
    std::vector<double> spd(size_t(3 + kThermoCoef) * ns);
    for (int k = 0; k < ns; k++) {
        spd[k] = hm.W[k];
        spd[size_t(ns) + k] = 1.0 / hm.W[k];
        spd[size_t(2) * ns + k] = hm.Tmid[k];
        for (int rg = 0; rg < 2; rg++) {
            const double *a = rg == 0 ? &hm.alow[7 * k] : &hm.ahigh[7 * k];
            double c[21] = {a[0], a[1], a[2], a[3], a[4],
                            a[0], a[1] / 2.0, a[2] / 3.0, a[3] / 4.0, a[4] / 5.0, a[5],
                            a[0], a[1], a[2] / 2.0, a[3] / 3.0, a[4] / 4.0, a[6],
                            a[1], 2.0 * a[2], 3.0 * a[3], 4.0 * a[4]};
            for (int j = 0; j < 21; j++) spd[size_t(3 + 21 * rg + j) * ns + k] = c[j];
        }
    }
    // Reactions sorted by type (stable), the most complex first, and within a type by species slot
    // count, the fewest first: the kernels hand consecutive blocks of 64 reactions to the lanes of
    // a wavefront, and a block pays for the most complex type it holds and loops over its largest
    // slot count.  So the few third-body and fall-off reactions share the leading blocks, topped up
    // with the smallest elementary reactions, and the ragged last block holds elementary ones only.
    std::vector<int> order(nr);
    std::iota(order.begin(), order.end(), 0);
    auto slots = [&](int i) { return hm.rx[i].rsp.size() + hm.rx[i].psp.size(); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (hm.rx[a].type != hm.rx[b].type) return hm.rx[a].type > hm.rx[b].type;
        return slots(a) < slots(b);
    });
    std::vector<RxnRec> rx(std::max(nr, 1));
    std::vector<FallRec> fall;
    std::vector<EffRec> eff;
    std::vector<int> orig(std::max(nr, 1));
    for (int ii = 0; ii < nr; ii++) {
        const auto &x = hm.rx[order[ii]];
        RxnRec &R = rx[ii];
        std::memset(&R, 0, sizeof(R));
        orig[ii] = order[ii];
        R.lnA = std::log(x.A);
        R.beta = x.beta;
        R.EaR = x.Ea / hm.R;
        int s = 0, nu = 0, sp[6] = {0, 0, 0, 0, 0, 0};
        double d = 0;
        for (size_t j = 0; j < x.rsp.size(); j++, s++) {
            sp[s] = x.rsp[j];
            nu |= x.rnu[j] << (2 * s);
            d -= x.rnu[j];
        }
        const int nre = s;
        for (size_t j = 0; j < x.psp.size(); j++, s++) {
            sp[s] = x.psp[j];
            nu |= x.pnu[j] << (2 * s);
            d += x.pnu[j];
        }
        R.dnu = d;
        R.meta = (x.type & 3) | ((x.rev ? 1 : 0) << 2) | (s << 3) | (nre << 6) | (int(x.eff.size()) << 9);
        R.eff_begin = int(eff.size());
        for (int j = 0; j < 3; j++) R.sp[j] = sp[2 * j] | (sp[2 * j + 1] << 16);
        R.nu = nu;
        R.fall = -1;
        if (x.type >= 2) {
            FallRec F{};
            F.lnA0 = std::log(x.A0);
            F.beta0 = x.beta0;
            F.Ea0R = x.Ea0 / hm.R;
            if (x.type == 3) {
                F.a = x.ta;
                F.invT3 = 1.0 / x.T3;
                F.invT1 = 1.0 / x.T1;
                F.T2 = x.T2;
            }
            R.fall = int(fall.size());
            fall.push_back(F);
        }
        for (auto &e : x.eff) {
            EffRec E{};
            E.am1 = e.second - 1.0;
            E.sp = e.first;
            eff.push_back(E);
        }
    }
    for (int b0 = 0; b0 < nr; b0 += 64) {
        int mx = 0;
        for (int i = b0; i < std::min(nr, b0 + 64); i++) mx = std::max(mx, rx_nslot(rx[i].meta));
        for (int i = b0; i < std::min(nr, b0 + 64); i++) rx[i].blk_slots = mx;
    }
    if (fall.empty()) fall.resize(1);
    if (eff.empty()) eff.resize(1);

    Packer pk;
    const size_t ospd = pk.add(spd), orx = pk.add(rx), ofall = pk.add(fall), oeff = pk.add(eff), oorig = pk.add(orig);

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
    d.n_eff = int(eff.size());
    d.R = hm.R;
    d.ln_p0_R = std::log(hm.p0 / hm.R);
    d.spd = reinterpret_cast<const double *>(b + ospd);
    d.rx = reinterpret_cast<const RxnRec *>(b + orx);
    d.fall = reinterpret_cast<const FallRec *>(b + ofall);
    d.eff = reinterpret_cast<const EffRec *>(b + oeff);
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
    for (auto &w : m->ws)
        if (w.ptr) hipFree(w.ptr);
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
