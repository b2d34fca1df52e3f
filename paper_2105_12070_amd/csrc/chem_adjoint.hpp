// Discrete adjoint of the Rosenbrock integration (device side).
#pragma once
#include "chem_cell.hpp"
