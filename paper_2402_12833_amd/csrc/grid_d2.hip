// Structured-grid solver, bulk type double, 2D.
#include "solver_grid.hpp"

namespace amg {

SolverBase* new_grid_solver_d2(const amgmpcg_grid& g, const amgmpcg_options& o, hipStream_t s,
                                  const double* st9) {
    return new Solver<double, 2>(g, o, s, st9);
}

}  // namespace amg
