// Per-family dispatch: kernel parameter blocks and launches.
#include "families.h"

namespace pvi {

static int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

ADev make_adev(const pvi_mdp* p) {
    ADev a{};
    const int R = p->rad[0];
    a.R = R;
    a.m = p->m;
    a.dmax = p->dmax[0];
    a.xt = p->xt;
    a.tab = p->tab;
    a.nz = p->m >= 2 ? (int)ipow(R, p->m - 2) : 1;
    a.r2 = p->m >= 2 ? R : 1;
    a.tiles = (int)(ipow(R, p->L - 1) * a.nz);
    a.stride_a = ipow(R, p->m + p->L - 2);
    a.stride_h = ipow(R, p->m - 1);
    for (int i = 0; i < 8; ++i) a.pow_y[i] = (int)ipow(R, i);
    a.gamma = p->d.gamma;
    a.cvar = p->d.c_var[0];
    a.pmf = p->dev.pmf;
    a.cdf = p->dev.cdf;
    a.tail = p->dev.tail;
    a.r0 = p->dev.r0;
    a.ctl = p->dev.ctl;
    a.partials = p->dev.partials;
    a.pi = p->dev.pi;
    a.gap = p->dev.gap;
    return a;
}

bool family_supported(const pvi_mdp* p) { return p->family == PVI_FAMILY_LEADTIME; }

std::string family_support_msg(const pvi_mdp* p) {
    if (family_supported(p)) return "ok";
    return "this family has no GPU kernel yet";
}

int family_tiles(const pvi_mdp* p) {
    if (p->family == PVI_FAMILY_LEADTIME) {
        const int R = p->rad[0];
        return (int)(ipow(R, p->L - 1) * (p->m >= 2 ? ipow(R, p->m - 2) : 1));
    }
    return 1;
}

size_t family_extra_bytes(const pvi_mdp* p) {
    if (p->family == PVI_FAMILY_LEADTIME)
        return sizeof(double) * (3 * (size_t)p->tab + p->a_r0.size());
    return 0;
}

pvi_status family_init(pvi_mdp*) { return PVI_OK; }

void family_free(pvi_mdp*) {}

hipError_t family_backup(pvi_mdp* p, int fp32, int kahan, int extract, const void* vin,
                         void* vout, hipStream_t s) {
    if (p->family == PVI_FAMILY_LEADTIME) {
        ADev a = make_adev(p);
        a.v_in = vin;
        a.v_out = vout;
        return launch_backup_a(a, fp32, kahan, extract, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace pvi
