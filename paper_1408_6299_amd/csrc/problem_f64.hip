// Problem handles with double transport: instantiates every kernel they launch.
#include "problem.hpp"

namespace nk {

ProblemBase* make_problem_f64(const nkreg_config& c, hipStream_t s) { return new ProblemT<double>(c, s); }

}  // namespace nk
