// Checkpoint files: the value tables a solve needs to go on (the last V, and under
// the periodic rule the tables its test reads), the FP64 sweep count, and a
// fingerprint of the MDP, so a solve cut short (the paper restarts interrupted
// cloud sessions from its checkpoints) resumes where it stopped.
#include "checkpoint.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "pvi_internal.h"

namespace pvi {

namespace {

constexpr char kMagic[8] = {'P', 'V', 'I', 'C', 'K', 'P', 'T', '1'};
constexpr uint32_t kVersion = 2;  // version 1 (no threshold or increments) is still read
constexpr int kMaxTables = PVI_MAX_PERIODS + 1;

struct Header {
    char magic[8];
    uint32_t version, family;
    uint64_t fingerprint;
    int64_t ns;
    int32_t na, rule, sweeps, stopped, hist, reserved;
};
static_assert(sizeof(Header) == 56, "checkpoint header layout");
// follows the header in version 2
struct HeaderStats {
    double threshold, dmax, dmin, span;
};
static_assert(sizeof(HeaderStats) == 32, "checkpoint header layout");

struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void bytes(const void* q, size_t n) {
        const unsigned char* c = static_cast<const unsigned char*>(q);
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
    }
    template <class T>
    void val(const T& v) {
        bytes(&v, sizeof v);
    }
    void vec(const std::vector<double>& v) {
        val((uint64_t)v.size());
        if (!v.empty()) bytes(v.data(), sizeof(double) * v.size());
    }
};

struct File {
    FILE* f = nullptr;
    ~File() {
        if (f) std::fclose(f);
    }
};

}  // namespace

uint64_t mdp_fingerprint(const pvi_mdp* p) {
    Fnv h;
    for (int v : {p->family, p->m, p->L, p->P, p->rad[0], p->rad[1], p->dmax[0], p->dmax[1],
                  p->na, (int)p->d.issuing})
        h.val((int32_t)v);
    h.val((int64_t)p->ns);
    for (double v : {p->d.gamma, p->d.subst_rho, p->d.c_var[0], p->d.c_var[1], p->d.c_fixed,
                     p->d.c_hold, p->d.c_short, p->d.c_waste, p->d.c_rev[0], p->d.c_rev[1]})
        h.val(v);
    h.vec(p->pmf[0]);
    h.vec(p->pmf[1]);
    h.vec(p->life);
    return h.h;
}

pvi_status checkpoint_load(const pvi_mdp* p, const char* path, bool want_tables,
                           Checkpoint& out) {
    const std::string w = std::string("checkpoint ") + (path ? path : "(null)");
    if (!path) return fail(PVI_E_INVALID, "checkpoint: NULL path");
    File in;
    in.f = std::fopen(path, "rb");
    if (!in.f) return fail(PVI_E_IO, w + ": cannot open");
    Header hd{};
    if (std::fread(&hd, sizeof hd, 1, in.f) != 1) return fail(PVI_E_IO, w + ": short header");
    if (std::memcmp(hd.magic, kMagic, sizeof kMagic) != 0)
        return fail(PVI_E_INVALID, w + ": not a checkpoint file");
    if (hd.version != 1 && hd.version != kVersion)
        return fail(PVI_E_INVALID, w + ": unknown version");
    if (hd.fingerprint != mdp_fingerprint(p) || hd.ns != p->ns || hd.na != p->na ||
        (int)hd.family != p->family)
        return fail(PVI_E_INVALID, w + ": written for another MDP descriptor");
    if (hd.hist < 1 || hd.hist > kMaxTables || hd.sweeps < 0 || (hd.stopped & ~1) != 0 ||
        hd.rule < PVI_STOP_SPAN || hd.rule > PVI_STOP_PERIODIC)
        return fail(PVI_E_INVALID, w + ": corrupt header");
    HeaderStats hs{std::nan(""), 0.0, 0.0, 0.0};
    if (hd.version >= 2 && std::fread(&hs, sizeof hs, 1, in.f) != 1)
        return fail(PVI_E_IO, w + ": short header");
    out.rule = hd.rule;
    out.sweeps = hd.sweeps;
    out.stopped = hd.stopped;
    out.threshold = hs.threshold;
    out.dmax = hs.dmax;
    out.dmin = hs.dmin;
    out.span = hs.span;
    out.tables.clear();
    const int n = want_tables ? hd.hist : 1;
    for (int k = 0; k < n; ++k) {
        std::vector<double> t((size_t)p->ns);
        if (std::fread(t.data(), sizeof(double), t.size(), in.f) != t.size())
            return fail(PVI_E_IO, w + ": short value table");
        out.tables.push_back(std::move(t));
    }
    if (want_tables) {
        unsigned char extra;
        if (std::fread(&extra, 1, 1, in.f) != 0)
            return fail(PVI_E_INVALID, w + ": trailing bytes");
    }
    return PVI_OK;
}

pvi_status checkpoint_store(const pvi_mdp* p, const char* path, int32_t rule, int32_t sweeps,
                            int32_t stopped, const CheckpointStats& stats,
                            const double* const* tables, int n_tables, hipStream_t s) {
    if (!path || n_tables < 1 || n_tables > kMaxTables)
        return fail(PVI_E_INVALID, "checkpoint: bad arguments");
    std::vector<double> host((size_t)n_tables * p->ns);
    for (int k = 0; k < n_tables; ++k)
        PVI_HIP(hipMemcpyAsync(host.data() + (size_t)k * p->ns, tables[k],
                               sizeof(double) * p->ns, hipMemcpyDeviceToHost, s));
    PVI_HIP(hipStreamSynchronize(s));
    Header hd{};
    std::memcpy(hd.magic, kMagic, sizeof kMagic);
    hd.version = kVersion;
    hd.family = (uint32_t)p->family;
    hd.fingerprint = mdp_fingerprint(p);
    hd.ns = p->ns;
    hd.na = p->na;
    hd.rule = rule;
    hd.sweeps = sweeps;
    hd.stopped = stopped ? 1 : 0;
    hd.hist = n_tables;
    const HeaderStats hs{stats.threshold, stats.dmax, stats.dmin, stats.span};
    const std::string tmp = std::string(path) + ".tmp";
    {
        File o;
        o.f = std::fopen(tmp.c_str(), "wb");
        if (!o.f) return fail(PVI_E_IO, "checkpoint " + tmp + ": cannot create");
        if (std::fwrite(&hd, sizeof hd, 1, o.f) != 1 || std::fwrite(&hs, sizeof hs, 1, o.f) != 1 ||
            std::fwrite(host.data(), sizeof(double), host.size(), o.f) != host.size() ||
            std::fflush(o.f) != 0)
            return fail(PVI_E_IO, "checkpoint " + tmp + ": write failed");
        const int rc = std::fclose(o.f);
        o.f = nullptr;
        if (rc != 0) return fail(PVI_E_IO, "checkpoint " + tmp + ": write failed");
    }
    if (std::rename(tmp.c_str(), path) != 0)
        return fail(PVI_E_IO, std::string("checkpoint ") + path + ": rename failed");
    return PVI_OK;
}

}  // namespace pvi

extern "C" pvi_status checkpoint_read(const pvi_mdp* mdp, const char* path, double* v,
                                      int32_t* sweeps, int32_t* stopped) {
    if (!mdp) return pvi::fail(PVI_E_INVALID, "checkpoint_read: NULL handle");
    pvi::Checkpoint c;
    const pvi_status st = pvi::checkpoint_load(mdp, path, false, c);
    if (st != PVI_OK) return st;
    if (v) std::memcpy(v, c.tables[0].data(), sizeof(double) * mdp->ns);
    if (sweeps) *sweeps = c.sweeps;
    if (stopped) *stopped = c.stopped;
    return PVI_OK;
}
