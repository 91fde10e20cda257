// Vector kernels of the CG solvers (placeholder unit; filled by the solver).
#include "kernels.hpp"
