// Host-side policy of the refinement that solves B t = g for the correction
// vector of eq. compv (t = (A D W)^+ g, B = A D W): which candidate t to keep,
// and whether to take another step, build a better approximate
// pseudo-inverse, or stop.  Plain C++ without HIP, so that the policy is
// exercised on its own on the CPU.
#pragma once

#include <cmath>

namespace skipm {

struct VRefine {
  double target = 1e-14;  // ||B t - g|| / ||g|| that ends the refinement
  int max_steps = 12;
  int max_round = 2;      // approximate pseudo-inverses: round 0 (B^T Q^{-1}), 1, 2 (whitened)
  double best = 1.0;      // relative residual of the kept t (t = 0 at the start: 1)
  int round = 0;          // round the next step uses
  int steps = 0;
};

enum VAct { V_STOP = 0, V_NEXT = 1, V_BUILD = 2 };

// One refinement step produced a candidate t' = t + P (g - B t) whose relative
// residual is rel (NaN or inf if the arithmetic broke down).  *keep: whether t'
// replaces the kept t (only a finite residual strictly below the kept one
// does, so the kept t never gets worse and never turns non-finite).  Returns
// V_STOP when the target is met, the step budget is spent, or no better
// pseudo-inverse is left to try while the last step contracted by less than
// half; V_BUILD when the step contracted by less than 1e-2 (or failed) and a
// further round exists (round is advanced: build it, then step again);
// V_NEXT otherwise.
inline VAct v_refine_next(VRefine& s, double rel, bool* keep) {
  ++s.steps;
  const bool ok = std::isfinite(rel) && rel >= 0.0;
  *keep = ok && rel < s.best;
  const double ratio = ok ? rel / s.best : HUGE_VAL;  // contraction against the kept t
  if (*keep) s.best = rel;
  if (!(s.best > s.target) || s.steps >= s.max_steps) return V_STOP;
  if (s.round < s.max_round && ratio > 1e-2) {
    ++s.round;
    return V_BUILD;
  }
  if (ratio > 0.5) return V_STOP;  // stagnated at the attainable accuracy
  return V_NEXT;
}

}  // namespace skipm
