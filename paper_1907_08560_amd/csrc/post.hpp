// post.hpp -- outputs of the sweeps (lambda, X).
#pragma once

#include "solver.hpp"
