// Circuit front end: OpenQASM 2.0 parsing and gate fusion (Sec. III: the
// simulator reads OpenQASM and fuses the circuit into one- and two-qubit
// gates before applying it; Sec. IV.A: sequential gates that share qubits
// are compressed to reduce the number of contractions).
//
// Host code only.  Gate matrices follow the standard definitions:
//   U(t, p, l) = [[cos(t/2), -e^{il} sin(t/2)], [e^{ip} sin(t/2), e^{i(p+l)} cos(t/2)]],
//   R_P(t) = exp(-i t P / 2), p(l) = u1(l) = diag(1, e^{il}),
// a controlled gate acts with its first argument as control, and a two-qubit
// matrix has row 2*s_q0 + s_q1 (q0 = first argument).
#include <array>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/tnsim.h"

namespace {

using cd = std::complex<double>;
constexpr double kPi = 3.14159265358979323846;
using M2 = std::array<cd, 4>;
using M4 = std::array<cd, 16>;

struct QasmError {
  std::string msg;
};

[[noreturn]] void fail_at(int line, const std::string &m) {
  throw QasmError{"line " + std::to_string(line) + ": " + m};
}

// ------------------------------------------------------------------ tokens
struct Tok {
  enum Kind { ID, NUM, STR, SYM, END } k;
  std::string s;
  double v = 0.0;
  int line = 0;
};

std::vector<Tok> lex(const char *text) {
  std::vector<Tok> out;
  int line = 1;
  const char *p = text;
  while (*p) {
    const char c = *p;
    if (c == '\n') {
      line++;
      p++;
    } else if (isspace((unsigned char)c)) {
      p++;
    } else if (c == '/' && p[1] == '/') {
      while (*p && *p != '\n') p++;
    } else if (c == '/' && p[1] == '*') {
      p += 2;
      while (*p && !(p[0] == '*' && p[1] == '/')) line += (*p++ == '\n');
      if (!*p) fail_at(line, "unterminated comment");
      p += 2;
    } else if (isalpha((unsigned char)c) || c == '_') {
      const char *b = p;
      while (isalnum((unsigned char)*p) || *p == '_') p++;
      out.push_back({Tok::ID, std::string(b, p), 0.0, line});
    } else if (isdigit((unsigned char)c) || (c == '.' && isdigit((unsigned char)p[1]))) {
      char *e = nullptr;
      const double v = strtod(p, &e);
      out.push_back({Tok::NUM, std::string((const char *)p, (const char *)e), v, line});
      p = e;
    } else if (c == '"') {
      const char *b = ++p;
      while (*p && *p != '"' && *p != '\n') p++;
      if (*p != '"') fail_at(line, "unterminated string");
      out.push_back({Tok::STR, std::string(b, p), 0.0, line});
      p++;
    } else if ((c == '-' && p[1] == '>') || (c == '=' && p[1] == '=')) {
      out.push_back({Tok::SYM, std::string(p, 2), 0.0, line});
      p += 2;
    } else if (strchr(";,()[]{}+-*/^", c)) {
      out.push_back({Tok::SYM, std::string(1, c), 0.0, line});
      p++;
    } else {
      fail_at(line, std::string("unexpected character '") + c + "'");
    }
  }
  out.push_back({Tok::END, "", 0.0, line});
  return out;
}

// ------------------------------------------------------------------ gate matrices
M2 u3(double t, double ph, double l) {
  const double c = std::cos(t / 2), s = std::sin(t / 2);
  return {cd(c, 0), -std::polar(1.0, l) * s, std::polar(1.0, ph) * s, std::polar(1.0, ph + l) * c};
}
M2 rot(char axis, double t) {
  const double c = std::cos(t / 2), s = std::sin(t / 2);
  const cd mi(0, -1);
  if (axis == 'x') return {cd(c, 0), mi * s, mi * s, cd(c, 0)};
  if (axis == 'y') return {cd(c, 0), cd(-s, 0), cd(s, 0), cd(c, 0)};
  return {std::polar(1.0, -t / 2), 0.0, 0.0, std::polar(1.0, t / 2)};
}
M2 phase(double l) { return {1.0, 0.0, 0.0, std::polar(1.0, l)}; }
M2 mat2(cd a, cd b, cd c, cd d) { return {a, b, c, d}; }

M4 controlled(const M2 &u) {
  M4 m{};
  m[0] = m[5] = 1.0;
  m[10] = u[0];
  m[11] = u[1];
  m[14] = u[2];
  m[15] = u[3];
  return m;
}
// exp(-i t/2 P(x)P) for P in {X, Y, Z}
M4 pauli_pair(char axis, double t) {
  M2 p;
  if (axis == 'x') p = {0.0, 1.0, 1.0, 0.0};
  else if (axis == 'y') p = {0.0, cd(0, -1), cd(0, 1), 0.0};
  else p = {1.0, 0.0, 0.0, -1.0};
  M4 m{};
  const double c = std::cos(t / 2), s = std::sin(t / 2);
  for (int r = 0; r < 4; r++)
    for (int k = 0; k < 4; k++) {
      const cd pp = p[(r >> 1) * 2 + (k >> 1)] * p[(r & 1) * 2 + (k & 1)];
      m[r * 4 + k] = (r == k ? cd(c, 0) : cd(0, 0)) + cd(0, -s) * pp;
    }
  return m;
}

// ------------------------------------------------------------------ parser
struct GateDef {
  std::vector<std::string> params, args;
  size_t body_begin = 0, body_end = 0;  // token range of the body (between braces)
};

struct Parser {
  std::vector<Tok> t;
  size_t i = 0;
  std::map<std::string, std::pair<int, int>> qregs;  // name -> (offset, size)
  int nq = 0;
  std::map<std::string, int> cregs;
  std::map<std::string, GateDef> defs;
  std::vector<tnsim_gate> out;
  int depth = 0;

  const Tok &peek() const { return t[i]; }
  const Tok &next() { return t[i++]; }
  bool is_sym(const char *s) const { return t[i].k == Tok::SYM && t[i].s == s; }
  bool is_id(const char *s) const { return t[i].k == Tok::ID && t[i].s == s; }
  void expect_sym(const char *s) {
    if (!is_sym(s)) fail_at(peek().line, std::string("expected '") + s + "'");
    i++;
  }
  std::string expect_id() {
    if (peek().k != Tok::ID) fail_at(peek().line, "expected a name");
    return next().s;
  }
  int expect_int() {
    const Tok &k = next();
    if (k.k != Tok::NUM || k.v != std::floor(k.v) || k.v < 0 || k.v > 1e7)
      fail_at(k.line, "expected a non-negative integer");
    return (int)k.v;
  }

  // expressions over the parameters in scope
  double expr(const std::map<std::string, double> &env) {
    double v = term(env);
    while (is_sym("+") || is_sym("-")) {
      const bool plus = next().s == "+";
      const double r = term(env);
      v = plus ? v + r : v - r;
    }
    return v;
  }
  double term(const std::map<std::string, double> &env) {
    double v = power(env);
    while (is_sym("*") || is_sym("/")) {
      const bool mul = next().s == "*";
      const double r = power(env);
      v = mul ? v * r : v / r;
    }
    return v;
  }
  double power(const std::map<std::string, double> &env) {
    const double b = unary(env);
    if (is_sym("^")) {
      i++;
      return std::pow(b, power(env));
    }
    return b;
  }
  int nest = 0;  // expression nesting, bounded so that a hostile text cannot exhaust the stack
  double unary(const std::map<std::string, double> &env) {
    struct Guard {
      int &n;
      Guard(int &x, int line) : n(x) {
        if (++n > 256) fail_at(line, "expression nested too deeply");
      }
      ~Guard() { n--; }
    } guard(nest, peek().line);
    if (is_sym("-")) {
      i++;
      return -unary(env);
    }
    if (is_sym("+")) {
      i++;
      return unary(env);
    }
    return primary(env);
  }
  double primary(const std::map<std::string, double> &env) {
    const Tok &k = next();
    if (k.k == Tok::NUM) return k.v;
    if (k.k == Tok::SYM && k.s == "(") {
      const double v = expr(env);
      expect_sym(")");
      return v;
    }
    if (k.k == Tok::ID) {
      if (k.s == "pi") return kPi;
      auto it = env.find(k.s);
      if (it != env.end()) return it->second;
      static const std::map<std::string, double (*)(double)> fn = {
          {"sin", std::sin}, {"cos", std::cos}, {"tan", std::tan},
          {"exp", std::exp}, {"ln", std::log},  {"sqrt", std::sqrt}};
      auto f = fn.find(k.s);
      if (f != fn.end()) {
        expect_sym("(");
        const double v = expr(env);
        expect_sym(")");
        return f->second(v);
      }
      fail_at(k.line, "unknown parameter '" + k.s + "'");
    }
    fail_at(k.line, "bad expression");
  }

  void emit1(int q, const M2 &m) {
    tnsim_gate g;
    memset(&g, 0, sizeof g);
    g.q0 = q;
    g.q1 = -1;
    for (int k = 0; k < 4; k++) g.m[k] = {m[k].real(), m[k].imag()};
    out.push_back(g);
  }
  void emit2(int a, int b, const M4 &m, int line) {
    if (a == b) fail_at(line, "a two-qubit gate needs two different qubits");
    tnsim_gate g;
    memset(&g, 0, sizeof g);
    g.q0 = a;
    g.q1 = b;
    for (int k = 0; k < 16; k++) g.m[k] = {m[k].real(), m[k].imag()};
    out.push_back(g);
  }

  // a built-in gate on resolved qubits; false if the name is not built in
  bool builtin(const std::string &n, const std::vector<double> &p, const std::vector<int> &q,
               int line) {
    auto need = [&](size_t np, size_t nq) {
      if (p.size() != np) fail_at(line, "gate '" + n + "' takes " + std::to_string(np) + " parameters");
      if (q.size() != nq) fail_at(line, "gate '" + n + "' takes " + std::to_string(nq) + " qubits");
    };
    const double r2 = std::sqrt(0.5);
    const cd I(0, 1);
    static const std::map<std::string, int> one = {
        {"id", 0}, {"i", 0}, {"x", 1}, {"y", 2}, {"z", 3}, {"h", 4}, {"s", 5}, {"sdg", 6},
        {"t", 7}, {"tdg", 8}, {"sx", 9}, {"sxdg", 10}};
    auto fixed1 = [&](int k) -> M2 {
      switch (k) {
        case 0: return mat2(1.0, 0.0, 0.0, 1.0);
        case 1: return mat2(0.0, 1.0, 1.0, 0.0);
        case 2: return mat2(0.0, -I, I, 0.0);
        case 3: return mat2(1.0, 0.0, 0.0, -1.0);
        case 4: return mat2(r2, r2, r2, -r2);
        case 5: return phase(kPi / 2);
        case 6: return phase(-kPi / 2);
        case 7: return phase(kPi / 4);
        case 8: return phase(-kPi / 4);
        case 9: return mat2(cd(0.5, 0.5), cd(0.5, -0.5), cd(0.5, -0.5), cd(0.5, 0.5));
        default: return mat2(cd(0.5, -0.5), cd(0.5, 0.5), cd(0.5, 0.5), cd(0.5, -0.5));
      }
    };
    auto f1 = one.find(n);
    if (f1 != one.end()) {
      need(0, 1);
      emit1(q[0], fixed1(f1->second));
      return true;
    }
    if (n == "rx" || n == "ry" || n == "rz") {
      need(1, 1);
      emit1(q[0], rot(n[1], p[0]));
    } else if (n == "p" || n == "u1") {
      need(1, 1);
      emit1(q[0], phase(p[0]));
    } else if (n == "u2") {
      need(2, 1);
      emit1(q[0], u3(kPi / 2, p[0], p[1]));
    } else if (n == "u3" || n == "u" || n == "U") {
      need(3, 1);
      emit1(q[0], u3(p[0], p[1], p[2]));
    } else if (n == "cx" || n == "CX" || n == "cy" || n == "cz" || n == "ch" || n == "csx") {
      need(0, 2);
      const int k = n == "cy" ? 2 : n == "cz" ? 3 : n == "ch" ? 4 : n == "csx" ? 9 : 1;
      emit2(q[0], q[1], controlled(fixed1(k)), line);
    } else if (n == "crx" || n == "cry" || n == "crz") {
      need(1, 2);
      emit2(q[0], q[1], controlled(rot(n[2], p[0])), line);
    } else if (n == "cp" || n == "cu1") {
      need(1, 2);
      emit2(q[0], q[1], controlled(phase(p[0])), line);
    } else if (n == "cu3") {
      need(3, 2);
      emit2(q[0], q[1], controlled(u3(p[0], p[1], p[2])), line);
    } else if (n == "cu") {  // controlled U(t, p, l) with phase g on the control's |1>
      need(4, 2);
      M2 u = u3(p[0], p[1], p[2]);
      for (auto &x : u) x *= std::polar(1.0, p[3]);
      emit2(q[0], q[1], controlled(u), line);
    } else if (n == "swap") {
      need(0, 2);
      M4 m{};
      m[0] = m[6] = m[9] = m[15] = 1.0;
      emit2(q[0], q[1], m, line);
    } else if (n == "rxx" || n == "ryy" || n == "rzz") {
      need(1, 2);
      emit2(q[0], q[1], pauli_pair(n[1], p[0]), line);
    } else if (n == "ccx") {  // Toffoli by six CNOTs and T gates (Nielsen and Chuang Fig. 4.9)
      need(0, 3);
      const int a = q[0], b = q[1], c = q[2];
      const M4 cx = controlled(fixed1(1));
      if (a == b || b == c || a == c) fail_at(line, "ccx needs three different qubits");
      emit1(c, fixed1(4));
      emit2(b, c, cx, line);
      emit1(c, fixed1(8));
      emit2(a, c, cx, line);
      emit1(c, fixed1(7));
      emit2(b, c, cx, line);
      emit1(c, fixed1(8));
      emit2(a, c, cx, line);
      emit1(b, fixed1(7));
      emit1(c, fixed1(7));
      emit1(c, fixed1(4));
      emit2(a, b, cx, line);
      emit1(a, fixed1(7));
      emit1(b, fixed1(8));
      emit2(a, b, cx, line);
    } else if (n == "cswap") {  // Fredkin = CX(c,b) Toffoli(a,b,c) CX(c,b)
      need(0, 3);
      const M4 cx = controlled(fixed1(1));
      emit2(q[2], q[1], cx, line);
      builtin("ccx", {}, {q[0], q[1], q[2]}, line);
      emit2(q[2], q[1], cx, line);
    } else {
      return false;
    }
    return true;
  }

  // one statement at top level (scope == nullptr) or inside a gate body
  void statement(const std::map<std::string, double> *penv,
                 const std::map<std::string, int> *qenv) {
    const Tok &k = peek();
    if (k.k != Tok::ID) fail_at(k.line, "expected a statement");
    const std::string w = k.s;
    const int line = k.line;
    if (!qenv) {
      if (w == "OPENQASM") {
        i++;
        const Tok &v = next();
        if (v.k != Tok::NUM || v.v < 2.0 || v.v >= 3.0) fail_at(line, "only OpenQASM 2 is read");
        expect_sym(";");
        return;
      }
      if (w == "include") {
        i++;
        if (next().k != Tok::STR) fail_at(line, "include needs a file name");
        expect_sym(";");  // the standard gate library is built in
        return;
      }
      if (w == "qreg" || w == "creg") {
        i++;
        const std::string name = expect_id();
        expect_sym("[");
        const int size = expect_int();
        expect_sym("]");
        expect_sym(";");
        if (size < 1) fail_at(line, "empty register");
        if (qregs.count(name) || cregs.count(name)) fail_at(line, "register declared twice");
        if (w == "qreg") {
          qregs[name] = {nq, size};
          nq += size;
        } else {
          cregs[name] = size;
        }
        return;
      }
      if (w == "gate") {
        i++;
        const std::string name = expect_id();
        GateDef d;
        if (is_sym("(")) {
          i++;
          while (!is_sym(")")) {
            d.params.push_back(expect_id());
            if (is_sym(",")) i++;
          }
          i++;
        }
        while (!is_sym("{")) {
          d.args.push_back(expect_id());
          if (is_sym(",")) i++;
        }
        i++;
        d.body_begin = i;
        while (!is_sym("}")) {
          if (peek().k == Tok::END) fail_at(line, "unterminated gate body");
          i++;
        }
        d.body_end = i;
        i++;
        defs[name] = d;
        return;
      }
      if (w == "opaque" || w == "reset" || w == "if")
        fail_at(line, "'" + w + "' is not supported (unitary circuits only)");
      if (w == "measure") {  // sampling of all qubits happens after the circuit
        while (!is_sym(";")) {
          if (peek().k == Tok::END) fail_at(line, "expected ';'");
          i++;
        }
        i++;
        return;
      }
    }
    if (w == "barrier") {
      while (!is_sym(";")) {
        if (peek().k == Tok::END) fail_at(line, "expected ';'");
        i++;
      }
      i++;
      return;
    }
    // a gate application
    i++;
    std::vector<double> params;
    static const std::map<std::string, double> none;
    if (is_sym("(")) {
      i++;
      while (!is_sym(")")) {
        params.push_back(expr(penv ? *penv : none));
        if (!std::isfinite(params.back())) fail_at(line, "a gate parameter is not finite");
        if (is_sym(",")) i++;
        else if (!is_sym(")")) fail_at(line, "expected ',' or ')'");
      }
      i++;
    }
    // arguments: register[index], whole registers (top level), or gate arguments
    std::vector<std::vector<int>> args;
    while (!is_sym(";")) {
      const std::string r = expect_id();
      if (qenv) {
        auto it = qenv->find(r);
        if (it == qenv->end()) fail_at(line, "unknown gate argument '" + r + "'");
        args.push_back({it->second});
      } else {
        auto it = qregs.find(r);
        if (it == qregs.end()) fail_at(line, "unknown quantum register '" + r + "'");
        if (is_sym("[")) {
          i++;
          const int idx = expect_int();
          expect_sym("]");
          if (idx >= it->second.second) fail_at(line, "qubit index out of range");
          args.push_back({it->second.first + idx});
        } else {
          std::vector<int> all;
          for (int j = 0; j < it->second.second; j++) all.push_back(it->second.first + j);
          args.push_back(all);
        }
      }
      if (is_sym(",")) i++;
      else if (!is_sym(";")) fail_at(line, "expected ',' or ';'");
    }
    i++;
    size_t reps = 1;
    for (auto &a : args)
      if (a.size() > 1) {
        if (reps > 1 && a.size() != reps) fail_at(line, "registers of different sizes");
        reps = a.size();
      }
    for (size_t r = 0; r < reps; r++) {
      std::vector<int> q;
      for (auto &a : args) q.push_back(a.size() > 1 ? a[r] : a[0]);
      for (size_t x = 0; x < q.size(); x++)
        for (size_t y = x + 1; y < q.size(); y++)
          if (q[x] == q[y]) fail_at(line, "a gate uses one qubit twice");
      apply(w, params, q, line);
    }
  }

  void apply(const std::string &name, const std::vector<double> &p, const std::vector<int> &q,
             int line) {
    auto it = defs.find(name);
    if (it == defs.end()) {
      if (!builtin(name, p, q, line)) fail_at(line, "unknown gate '" + name + "'");
      return;
    }
    const GateDef &d = it->second;
    if (p.size() != d.params.size() || q.size() != d.args.size())
      fail_at(line, "gate '" + name + "' called with the wrong number of parameters or qubits");
    if (++depth > 64) fail_at(line, "gate definitions nested too deeply");
    std::map<std::string, double> penv;
    std::map<std::string, int> qenv;
    for (size_t k = 0; k < p.size(); k++) penv[d.params[k]] = p[k];
    for (size_t k = 0; k < q.size(); k++) qenv[d.args[k]] = q[k];
    const size_t save = i;
    i = d.body_begin;
    while (i < d.body_end) statement(&penv, &qenv);
    i = save;
    depth--;
  }

  void run() {
    while (peek().k != Tok::END) statement(nullptr, nullptr);
  }
};

// ------------------------------------------------------------------ fusion
M4 kron(const M2 &a, const M2 &b) {  // a on the major (first) qubit
  M4 m;
  for (int r = 0; r < 4; r++)
    for (int c = 0; c < 4; c++) m[r * 4 + c] = a[(r >> 1) * 2 + (c >> 1)] * b[(r & 1) * 2 + (c & 1)];
  return m;
}
M4 mul4(const M4 &a, const M4 &b) {
  M4 m{};
  for (int r = 0; r < 4; r++)
    for (int k = 0; k < 4; k++)
      for (int c = 0; c < 4; c++) m[r * 4 + c] += a[r * 4 + k] * b[k * 4 + c];
  return m;
}
M2 mul2(const M2 &a, const M2 &b) {
  return {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3], a[2] * b[0] + a[3] * b[2],
          a[2] * b[1] + a[3] * b[3]};
}
M4 swapped(const M4 &g) {  // the same gate with its two qubits named in the other order
  M4 m;
  for (int r = 0; r < 4; r++)
    for (int c = 0; c < 4; c++)
      m[r * 4 + c] = g[((r & 1) * 2 + (r >> 1)) * 4 + (c & 1) * 2 + (c >> 1)];
  return m;
}
M2 get2(const tnsim_gate &g) { return {cd(g.m[0].re, g.m[0].im), cd(g.m[1].re, g.m[1].im), cd(g.m[2].re, g.m[2].im), cd(g.m[3].re, g.m[3].im)}; }
M4 get4(const tnsim_gate &g) {
  M4 m;
  for (int k = 0; k < 16; k++) m[k] = cd(g.m[k].re, g.m[k].im);
  return m;
}
void put4(tnsim_gate &g, const M4 &m) {
  for (int k = 0; k < 16; k++) g.m[k] = {m[k].real(), m[k].imag()};
}
void put2(tnsim_gate &g, const M2 &m) {
  memset(g.m, 0, sizeof g.m);
  for (int k = 0; k < 4; k++) g.m[k] = {m[k].real(), m[k].imag()};
}

}  // namespace

extern "C" {

tnsim_status tnsim_qasm_parse(const char *text, tnsim_gate *gates, int32_t cap, int32_t *n_gates,
                              int32_t *n_qubits, char *err, int32_t err_len) {
  if (err && err_len > 0) err[0] = 0;
  if (!text || !n_gates || !n_qubits || cap < 0 || (cap > 0 && !gates)) return TNSIM_E_ARG;
  Parser P;
  try {
    P.t = lex(text);
    P.run();
  } catch (const QasmError &e) {
    if (err && err_len > 0) snprintf(err, (size_t)err_len, "%s", e.msg.c_str());
    return TNSIM_E_ARG;
  }
  *n_qubits = P.nq;
  *n_gates = (int32_t)P.out.size();
  if ((int64_t)P.out.size() > cap) return TNSIM_E_CAPACITY;
  if (!P.out.empty()) memcpy(gates, P.out.data(), sizeof(tnsim_gate) * P.out.size());
  return TNSIM_OK;
}

tnsim_status tnsim_fuse(const tnsim_gate *in, int32_t n_in, int32_t n_qubits, tnsim_gate *out,
                        int32_t *n_out) {
  if (n_in < 0 || n_qubits < 1 || !n_out || (n_in > 0 && (!in || !out))) return TNSIM_E_ARG;
  for (int32_t k = 0; k < n_in; k++) {
    const int a = in[k].q0, b = in[k].q1;
    if (a < 0 || a >= n_qubits || b < -1 || b >= n_qubits || a == b) return TNSIM_E_ARG;
  }
  std::vector<tnsim_gate> res;
  std::vector<M2> pend(n_qubits, M2{1.0, 0.0, 0.0, 1.0});
  std::vector<char> has_pend(n_qubits, 0);
  std::vector<int> last(n_qubits, -1);  // output index of the last two-qubit gate on the qubit
  for (int32_t k = 0; k < n_in; k++) {
    const tnsim_gate &g = in[k];
    if (g.q1 < 0) {
      const int q = g.q0;
      const M2 u = get2(g);
      if (last[q] >= 0) {  // nothing touched q since that gate: fold u into it from the left
        tnsim_gate &h = res[last[q]];
        const M2 id{1.0, 0.0, 0.0, 1.0};
        put4(h, mul4(h.q0 == q ? kron(u, id) : kron(id, u), get4(h)));
      } else {
        pend[q] = mul2(u, pend[q]);
        has_pend[q] = 1;
      }
      continue;
    }
    const int a = g.q0, b = g.q1;
    M4 G = get4(g);
    // one-qubit gates still waiting on a or b act first
    G = mul4(G, kron(pend[a], pend[b]));
    pend[a] = pend[b] = M2{1.0, 0.0, 0.0, 1.0};
    has_pend[a] = has_pend[b] = 0;
    const int l = last[a];
    if (l >= 0 && l == last[b]) {  // the previous gate on both qubits is on this same pair
      tnsim_gate &h = res[l];
      put4(h, mul4(h.q0 == a ? G : swapped(G), get4(h)));
      continue;
    }
    tnsim_gate o = g;
    put4(o, G);
    res.push_back(o);
    last[a] = last[b] = (int)res.size() - 1;
  }
  for (int q = 0; q < n_qubits; q++)
    if (has_pend[q]) {
      tnsim_gate o;
      memset(&o, 0, sizeof o);
      o.q0 = q;
      o.q1 = -1;
      put2(o, pend[q]);
      res.push_back(o);
    }
  *n_out = (int32_t)res.size();
  if (!res.empty()) memcpy(out, res.data(), sizeof(tnsim_gate) * res.size());
  return TNSIM_OK;
}

}  // extern "C"
