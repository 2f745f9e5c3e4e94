// Structured-grid solver, bulk type float, 2D.
#include "solver_grid.hpp"

namespace amg {

SolverBase* new_grid_solver_f2(const amgmpcg_grid& g, const amgmpcg_options& o, hipStream_t s,
                                  const double* st9) {
    return new Solver<float, 2>(g, o, s, st9);
}

}  // namespace amg
