// HIP kernels of the Euler step (gfx950, wave64): the shared parts and the
// per-cell and LDS-tile families.  The register-march and resident kernels
// live in euler_march2d.h, euler_march3d.h and euler_resident1d.h.
#pragma once

#include "euler_analytic.h"
#include "euler_common.h"
#include "euler_direct.h"
#include "euler_lds.h"
