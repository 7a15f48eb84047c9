// Request server (filled in below).
#include <hip/hip_runtime.h>

#include "runtime.hpp"

extern "C" {
int camp_serve_create(long long, int, camp_server**) { camp::set_error("not built"); return CAMP_EINVAL; }
int camp_serve_submit(camp_server*, camp_mech*, int, double*, const camp_env*, double, double, double,
                      const camp_opts*, int*, long long*) { return CAMP_EINVAL; }
int camp_serve_poll(camp_server*, long long, int*, int*, double*) { return CAMP_EINVAL; }
int camp_serve_wait(camp_server*, long long) { return CAMP_EINVAL; }
int camp_serve_progress(camp_server*, int*, int*) { return CAMP_EINVAL; }
void camp_serve_destroy(camp_server*) {}
}
