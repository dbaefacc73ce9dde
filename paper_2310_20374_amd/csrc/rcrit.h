// Opening angle and critical radius of every cell (Sect. 3.4.2): theta(M) from the
// cell's mass, r_crit = r_max / theta, and the walk's packed cell record.  Run after
// the gravity climb, either as a launch of its own or by the gravity walk's init pass.
#pragma once
#include "ncorp_internal.h"

namespace ncorp {

// theta(M) of Dehnen's relation (recalled from Dehnen 2002; the paper's text does not
// print it), solved with only + - * /:
//   theta^15 M = K^3 M_root (1 - theta)^6,  K = theta_min^5 / (1 - theta_min)^2
__device__ inline double theta_of_mass(double M, double Mroot, double tmin) {
    if (!(M < Mroot)) return tmin;
    double tm = tmin, um = 1.0 - tmin;
    double tm2 = tm * tm, tm4 = tm2 * tm2, tm5 = tm4 * tm;
    double um2 = um * um;
    double K = tm5 / um2;
    double K3 = K * K * K;
    double rhs0 = K3 * Mroot;
    double lo = tmin, hi = 1.0;
    for (int it = 0; it < 64; it++) {
        double mid = 0.5 * (lo + hi);
        double t2 = mid * mid, t4 = t2 * t2, t8 = t4 * t4;
        double t15 = t8 * t4 * t2 * mid;
        double u = 1.0 - mid, u2 = u * u, u4 = u2 * u2, u6 = u4 * u2;
        double g = t15 * M - rhs0 * u6;
        if (g <= 0.0) lo = mid; else hi = mid;
    }
    return lo;
}

struct RcritArgs {
    const double *c_mass, *c_rmax;
    double4 *gcell;                  // w <- r_crit
    double *c_theta;
    double theta_min;
    int theta_mode;                  // 1: constant theta_min
    const int32_t *c_count, *c_child, *c_nchild, *c_entry, *c_nent, *c_first;
    WCell *wg;
    const uint16_t *seg;             // batched: disk of every tree position, else nullptr
    const int32_t *disk_root;
};

inline RcritArgs rcrit_args(const Workspace &ws, const ncorp_params &prm) {
    RcritArgs R;
    R.c_mass = ws.c_mass; R.c_rmax = ws.c_rmax; R.gcell = ws.gcell; R.c_theta = ws.c_theta;
    R.theta_min = prm.theta_min; R.theta_mode = prm.theta_mode;
    R.c_count = ws.c_count; R.c_child = ws.c_child; R.c_nchild = ws.c_nchild;
    R.c_entry = ws.c_entry; R.c_nent = ws.c_nent; R.c_first = ws.c_first;
    R.wg = ws.wg;
    R.seg = ws.ndisks > 1 ? ws.seg : nullptr;
    R.disk_root = ws.disk_root;
    return R;
}

__device__ inline void rcrit_cell(const RcritArgs &R, int c) {
    // M_root: mass of the root of this cell's own tree (its disk's)
    const double Mroot = R.c_mass[R.seg ? R.disk_root[R.seg[R.c_first[c]]] : 0];
    const double th = R.theta_mode == 1 ? R.theta_min
                                        : theta_of_mass(R.c_mass[c], Mroot, R.theta_min);
    R.c_theta[c] = th;
    const double rc = R.c_rmax[c] / th;
    double4 g = R.gcell[c];
    g.w = rc;
    R.gcell[c] = g;
    WCell w;
    w.x = g.x; w.y = g.y; w.z = g.z; w.rcrit = rc;
    w.count = R.c_count[c]; w.child = R.c_child[c]; w.nchild = R.c_nchild[c];
    w.entry = R.c_entry[c]; w.nent = R.c_nent[c]; w.first = R.c_first[c];
    w.pad[0] = w.pad[1] = 0;
    R.wg[c] = w;
}

}  // namespace ncorp
