// Structured-grid solver, bulk type float, 3D.
#include "solver_grid.hpp"

namespace amg {

SolverBase* new_grid_solver_f3(const amgmpcg_grid& g, const amgmpcg_options& o, hipStream_t s,
                                  const double* st9) {
    return new Solver<float, 3>(g, o, s, st9);
}

}  // namespace amg
