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
    return tb;
  }();
  return tab;
}

// The even-odd half tables (see TabH) from the full ones.  The points and
// the modes are used as symmetric: only the first ceil(Q/2) points enter.
template <typename T, int N, int Q>
void fill_tabh(const double* x, const double* B, const double* D, TabH<T, N, Q>& tb) {
  constexpr int H = TabH<T, N, Q>::H, KE = EO<N>::KE, KO = EO<N>::KO;
  for (int i = 0; i < H; ++i) {
    tb.BE[i * KE] = static_cast<T>(0.5);
    tb.DE[i * KE] = static_cast<T>(0.0);
    tb.BO[i * KO] = static_cast<T>(-0.5 * x[i]);
    tb.DO[i * KO] = static_cast<T>(-0.5);
    for (int m = 1; m < KE; ++m) {
      tb.BE[i * KE + m] = static_cast<T>(B[i * N + 2 * m - 1]);
      tb.DE[i * KE + m] = static_cast<T>(D[i * N + 2 * m - 1]);
    }
    for (int m = 1; m < KO; ++m) {
      tb.BO[i * KO + m] = static_cast<T>(B[i * N + 2 * m]);
      tb.DO[i * KO + m] = static_cast<T>(D[i * N + 2 * m]);
    }
  }
}

template <typename T, int N, int Q>
const TabH<T, N, Q>& host_tabh() {
  static const TabH<T, N, Q> tab = [] {
    TabH<T, N, Q> tb{};
    std::vector<double> x(Q), w(Q), B(Q * N), D(Q * N);
    gll_points(Q, x.data(), w.data());
    modified_basis(N - 1, Q, x.data(), B.data(), D.data());
    fill_tabh<T, N, Q>(x.data(), B.data(), D.data(), tb);
    return tb;
  }();
  return tab;
}

template <typename T, int N, int Q>
const TabK<T, N, Q>& host_tabk() {
  static const TabK<T, N, Q> tab = [] {
    TabK<T, N, Q> tk{};
    tk.h = host_tabh<T, N, Q>();
    if constexpr (N <= kPtMaxN) tk.f = host_tab<T, N, Q>();
    return tk;
  }();
  return tab;
}

}  // namespace nk
