// Problem handles with float transport: instantiates every kernel they launch.
#include "problem.hpp"

namespace nk {

ProblemBase* make_problem_f32(const nkreg_config& c, hipStream_t s) { return new ProblemT<float>(c, s); }

}  // namespace nk
