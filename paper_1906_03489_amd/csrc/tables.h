// Host construction of the 1-D basis tables passed to the kernels by value.
#pragma once

#include <vector>

#include "engine.h"

namespace nk {

template <typename T, int N, int Q>
const Tab<T, N, Q>& host_tab() {
  static const Tab<T, N, Q> tab = [] {
    Tab<T, N, Q> tb{};
    std::vector<double> x(Q), w(Q), B(Q * N), D(Q * N);
    gll_points(Q, x.data(), w.data());
    modified_basis(N - 1, Q, x.data(), B.data(), D.data());
    for (int i = 0; i < Q * N; ++i) {
      tb.B[i] = static_cast<T>(B[i]);
      tb.D[i] = static_cast<T>(D[i]);
    }
    for (int i = 0; i < (Q + 1) / 2; ++i) tb.X[i] = static_cast<T>(-0.5 * x[i]);
    return tb;
  }();
  return tab;
}

}  // namespace nk
