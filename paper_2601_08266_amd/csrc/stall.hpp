// Stagnation rule of the restarted FGMRES (host code, no HIP): a restart cycle stalls when its
// starting residual is above 99.9 % of the previous cycle's; three stalled cycles in a row end
// the solve.  A cycle that makes progress resets the count.
#pragma once

namespace fsi {

// prev_beta < 0: first cycle.  Returns true when the solve should stop.
inline bool krylov_stagnated(double prev_beta, double beta, int &stalls)
{
    if (prev_beta >= 0.0 && beta > 0.999 * prev_beta) return ++stalls >= 3;
    stalls = 0;
    return false;
}

}  // namespace fsi
