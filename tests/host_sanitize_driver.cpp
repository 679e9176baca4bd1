// Test driver of libbse's host-side numerics (csrc/host_math.cpp), built by
// tests/test_host_sanitize.py with the address and undefined-behaviour
// sanitizers.  Reads one command per line on stdin and prints the results:
//   signs SEED L S                      -> L*S signs
//   weights N DT GAMMA                  -> N+1 weights
//   tridiag M K A[0..M) B[0..M-1)       -> K eigenvalues, then K vectors of M
//   fit NB NE OMEGA[NB*NE] V[NB]        -> "ok" eps_inv c[NE] w_k0[NB], or "err MESSAGE"
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "host_math.h"

int main() {
  std::string line;
  std::cout.precision(17);
  while (std::getline(std::cin, line)) {
    std::istringstream in(line);
    std::string cmd;
    if (!(in >> cmd)) continue;
    if (cmd == "signs") {
      unsigned long long seed;
      int L, S;
      in >> seed >> L >> S;
      std::vector<int8_t> xi((size_t)L * S);
      bse_host::stochastic_signs(seed, L, S, xi.data());
      for (auto v : xi) std::cout << (int)v << ' ';
      std::cout << '\n';
    } else if (cmd == "weights") {
      int n;
      double dt, g;
      in >> n >> dt >> g;
      std::vector<double> w(n + 1);
      bse_host::time_weights(n, dt, g, w.data());
      for (double v : w) std::cout << v << ' ';
      std::cout << '\n';
    } else if (cmd == "tridiag") {
      int m, k;
      in >> m >> k;
      std::vector<double> a(m), b(m > 1 ? m - 1 : 0);
      for (auto& v : a) in >> v;
      for (auto& v : b) in >> v;
      std::vector<double> theta;
      std::vector<std::vector<double>> vecs;
      bse_host::tridiag_lowest(a, b, m, k, theta, vecs);
      for (double v : theta) std::cout << v << ' ';
      std::cout << '\n';
      for (const auto& vec : vecs) {
        for (double v : vec) std::cout << v << ' ';
        std::cout << '\n';
      }
    } else if (cmd == "fit") {
      int nb, ne;
      in >> nb >> ne;
      std::vector<double> om((size_t)(nb > 0 ? nb : 0) * (ne > 0 ? ne : 0)), v(nb > 0 ? nb : 0);
      for (auto& x : om) in >> x;
      for (auto& x : v) in >> x;
      std::vector<double> c(ne > 0 ? ne : 1), wk(nb > 0 ? nb : 1);
      double e = 0;
      const char* msg = bse_host::fit_box_correction(nb, ne, om.data(), v.data(), &e, c.data(), wk.data());
      if (msg) {
        std::cout << "err " << msg << '\n';
      } else {
        std::cout << "ok " << e;
        for (int i = 0; i < ne; ++i) std::cout << ' ' << c[i];
        for (int i = 0; i < nb; ++i) std::cout << ' ' << wk[i];
        std::cout << '\n';
      }
    } else {
      std::cerr << "unknown command " << cmd << '\n';
      return 2;
    }
  }
  return 0;
}
