// BTE entry points (grid states, pair tables, collision, dynamics, ITA).
#include "../../include/ephx.h"
#include "api_common.h"

using namespace ephx;

extern "C" int ephx_grid_states(ephx_model*, const int*, int, int, int, double, double, int, int, int*, int32_t*,
                                int32_t*, double*, void*) {
    return guarded([&] { throw Error{EPHX_EUNSUPPORTED, "grid_states: not built yet"}; });
}
extern "C" int ephx_table_create(ephx_model*, const int*, int, const int32_t*, const int32_t*, int, double,
                                 ephx_table**, void*) {
    return guarded([&] { throw Error{EPHX_EUNSUPPORTED, "table_create: not built yet"}; });
}
extern "C" int ephx_table_destroy(ephx_table*) { return EPHX_OK; }
extern "C" int ephx_table_g2(ephx_table*, float*, double*, void*) {
    return guarded([&] { throw Error{EPHX_EUNSUPPORTED, "table_g2: not built yet"}; });
}
extern "C" int ephx_collision_setup(ephx_table*, const ephx_params*, const double*, void*) {
    return guarded([&] { throw Error{EPHX_EUNSUPPORTED, "collision_setup: not built yet"}; });
}
extern "C" int ephx_collision(ephx_table*, const double*, double*, void*) {
    return guarded([&] { throw Error{EPHX_EUNSUPPORTED, "collision: not built yet"}; });
}
extern "C" int ephx_dynamics(ephx_table*, const double*, double, int, int, double*, double*, void*) {
    return guarded([&] { throw Error{EPHX_EUNSUPPORTED, "dynamics: not built yet"}; });
}
extern "C" int ephx_collision_vjp(ephx_table*, const double*, const double*, double*, double*, void*) {
    return guarded([&] { throw Error{EPHX_EUNSUPPORTED, "collision_vjp: not built yet"}; });
}
extern "C" int ephx_dynamics_vjp(ephx_table*, const double*, double, int, int, const double*, double*, double*,
                                 void*) {
    return guarded([&] { throw Error{EPHX_EUNSUPPORTED, "dynamics_vjp: not built yet"}; });
}
extern "C" int ephx_mobility(ephx_table*, const ephx_params*, const double*, int, double*, double*, double*, void*) {
    return guarded([&] { throw Error{EPHX_EUNSUPPORTED, "mobility: not built yet"}; });
}
