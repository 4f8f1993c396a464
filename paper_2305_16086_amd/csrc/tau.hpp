// Truncation length of one half-edge, shared by every kernel that needs it so
// that all paths agree bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

namespace sc {

__device__ inline int odd_at_least(double f) {
  long long k = static_cast<long long>(ceil(f));
  if (k < 1) k = 1;
  if ((k & 1) == 0) ++k;
  return k > INT_MAX ? INT_MAX : static_cast<int>(k);
}

// L > 0: the uniform odd L.  Else Theorem 3.2 with Upsilon = Delta = 0 (Eq. 6):
// the smallest odd tau with lam^(tau+1) (1/d_i + 1/d_j - 2/(d_i d_j)) /
// (1 - lam^2) <= eps_tau, not yet capped.
__device__ inline int tau_uncapped(int L, double di, double dj, double eps_tau, double lam) {
  if (L > 0) return L;
  const double num = 1.0 / di + 1.0 / dj - 2.0 / (di * dj);
  const double f = ceil(log(num / (eps_tau * (1.0 - lam * lam))) / log(1.0 / lam) - 1.0);
  return odd_at_least(f);
}

// As tau_uncapped, capped at max_L (automatic lengths only; a fixed L is the caller's).
__device__ inline int tau_of(int L, double di, double dj, double eps_tau, double lam, int max_L) {
  const int t = tau_uncapped(L, di, dj, eps_tau, lam);
  return (L <= 0 && t > max_L) ? max_L : t;
}

}  // namespace sc
