// Mutation fuzzing of the OpenQASM parser and gate fusion (host code), built
// with AddressSanitizer and UndefinedBehaviorSanitizer by test_qasm_fuzz.py.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>
#include "tnsim.h"
int main(int argc, char **argv) {
  std::mt19937 rng(12345);
  const char *seeds[] = {
      "OPENQASM 2.0;\ninclude \"qelib1.inc\";\nqreg q[5];\ncreg c[5];\nh q;\ncx q[0],q[3];\nccx q[0],q[1],q[4];\nrz(-pi/4+2*0.5^2) q[2];\nmeasure q -> c;\n",
      "OPENQASM 2.0;\nqreg a[3];\ngate my(t,u) x,y { rx(t) x; cx x,y; ry(u/2) y; barrier x,y; }\nmy(0.3,sin(0.2)) a[0],a[2];\nu3(1,2,3) a;\ncswap a[0],a[1],a[2];\n",
      "OPENQASM 2.0;\nqreg q[2];\n/* c */ rxx(1) q[0],q[1]; // x\ncu(1,2,3,4) q[1],q[0];\n"};
  const char alphabet[] = "qra[]();,{}+-*/^0123456789.pie \n\"/*_xhcgt";
  std::vector<tnsim_gate> g(4096), f(4096);
  char err[256];
  long ok = 0, bad = 0;
  const long iters = argc > 1 ? atol(argv[1]) : 20000;
  for (long it = 0; it < iters; it++) {
    std::string s = seeds[it % 3];
    const int muts = 1 + rng() % 6;
    for (int m = 0; m < muts; m++) {
      const size_t pos = rng() % (s.size() + 1);
      switch (rng() % 3) {
        case 0: s.insert(pos, 1, alphabet[rng() % (sizeof alphabet - 1)]); break;
        case 1: if (pos < s.size()) s.erase(pos, 1 + rng() % 3); break;
        default: if (pos < s.size()) s[pos] = alphabet[rng() % (sizeof alphabet - 1)]; break;
      }
    }
    int32_t n = 0, nq = 0;
    tnsim_status st = tnsim_qasm_parse(s.c_str(), g.data(), (int32_t)g.size(), &n, &nq, err, sizeof err);
    if (st == TNSIM_OK) {
      ok++;
      int32_t nf = 0;
      if (nq > 0 && tnsim_fuse(g.data(), n, nq, f.data(), &nf) != TNSIM_OK) { printf("fuse failed\n"); return 1; }
      if (nf > n) { printf("fuse grew\n"); return 1; }
    } else {
      bad++;
    }
  }
  printf("ok %ld rejected %ld\n", ok, bad);
  return 0;
}
