// Elliptic-cell body of revolution (multi-cell accelerator cavity profile).
#include "geometry.h"

namespace dm {

std::unique_ptr<Body> make_elliptic_bor(const dm_geometry &) { return nullptr; }

}  // namespace dm
