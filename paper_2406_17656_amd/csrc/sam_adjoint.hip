// sam_adjoint.hip -- placeholder translation unit (adjoint kernels follow).
#include "sam_device.hpp"
#include "sam_kernels.hpp"
