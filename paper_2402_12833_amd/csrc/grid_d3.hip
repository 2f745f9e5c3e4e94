// Structured-grid solver, bulk type double, 3D.
#include "solver_grid.hpp"

namespace amg {

SolverBase* new_grid_solver_d3(const amgmpcg_grid& g, const amgmpcg_options& o, hipStream_t s,
                                  const double* st9) {
    return new Solver<double, 3>(g, o, s, st9);
}

}  // namespace amg
