// Route selection and the hybrid driver of Algorithm 2 (Section III-B).
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"

namespace ccmi {

int run_label(Call& c) {
    hipError_t e = launch_sv_init(c.parent, c.n, c.stream);
    if (e != hipSuccess) return hip_fail(e, "sv_init launch");
    if (c.stats) c.bytes += 4.0 * c.n;
    if (c.m == 0) return CC_OK;
    int route = CC_R1_SV;
    switch (c.opt.route) {
        case CC_ROUTE_SV_THETA: route = CC_R2_SV_THETA; break;
        default: route = CC_R1_SV; break;
    }
    if (c.stats) c.stats->route = route;
    SvInput in;
    in.soa = true;
    in.u = c.u;
    in.v = c.v;
    in.m = c.m;
    int t0 = c.timer->mark();
    int rc = run_sv(c, in, route, c.opt.theta, c.opt.max_passes);
    int t1 = c.timer->mark();
    if (c.stats) c.stats->ms_sv = c.timer->ms(t0, t1);
    return rc;
}

}  // namespace ccmi
