// gates.cpp -- gate validation, FP64 gate matrices, thread-local errors.
//
// X, Y, Z and H are the matrices of Sec. II.A; rotation and phase gates use
// the OpenQASM-2 definitions listed in include/hisv.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include "hisv_internal.h"

namespace hisv {

static thread_local std::string t_last_error;

hs_status fail(hs_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_last_error = buf;
  return code;
}

void clear_error() { t_last_error.clear(); }
const char* last_error() { return t_last_error.c_str(); }

bool kind_is_1q(int kind) { return kind >= HS_H && kind <= HS_U3; }
bool kind_is_2q(int kind) { return kind >= HS_CX && kind <= HS_SWAP; }

hs_status validate_gate(int n, const hs_gate& g, Gate* out) {
  if (g.q2 != 0) return fail(HS_E_ARG, "q2 must be 0 for gate kind %d", g.kind);
  if (kind_is_1q(g.kind)) {
    if (g.q1 != -1) return fail(HS_E_ARG, "one-qubit gate kind %d needs q1 = -1", g.kind);
    if (g.q0 < 0 || g.q0 >= n)
      return fail(HS_E_QUBIT_RANGE, "qubit %d outside [0, %d)", g.q0, n);
  } else if (kind_is_2q(g.kind)) {
    if (g.q0 < 0 || g.q0 >= n || g.q1 < 0 || g.q1 >= n)
      return fail(HS_E_QUBIT_RANGE, "qubits (%d, %d) outside [0, %d)", g.q0, g.q1, n);
    if (g.q0 == g.q1) return fail(HS_E_QUBIT_RANGE, "two-qubit gate on one qubit %d", g.q0);
  } else {
    return fail(HS_E_ARG, "unknown gate kind %d", g.kind);
  }
  for (int i = 0; i < 3; ++i)
    if (!isfinite(g.p[i])) return fail(HS_E_ARG, "non-finite gate parameter");
  out->kind = g.kind;
  out->q0 = g.q0;
  out->q1 = g.q1;
  for (int i = 0; i < 3; ++i) out->p[i] = g.p[i];
  return HS_OK;
}

// A gate as it enters a circuit: one- and two-qubit kinds are validated and
// appended; the three-qubit kinds are replaced by one- and two-qubit gates.
//   CCX(a, b, t) = H(t) CX(b,t) Tdg(t) CX(a,t) T(t) CX(b,t) Tdg(t) CX(a,t)
//                  T(b) T(t) H(t) CX(a,b) T(a) Tdg(b) CX(a,b)
//   (the standard exact Toffoli decomposition, in circuit order), and
//   CSWAP(c, x, y) = CX(y, x) CCX(c, x, y) CX(y, x).
hs_status expand_gate(int n, const hs_gate& g, std::vector<Gate>* out) {
  if (g.kind != HS_CCX && g.kind != HS_CSWAP) {
    Gate v;
    if (hs_status rc = validate_gate(n, g, &v)) return rc;
    out->push_back(v);
    return HS_OK;
  }
  const int a = g.q0, b = g.q1, c = g.q2;
  if (a < 0 || a >= n || b < 0 || b >= n || c < 0 || c >= n)
    return fail(HS_E_QUBIT_RANGE, "qubits (%d, %d, %d) outside [0, %d)", a, b, c, n);
  if (a == b || a == c || b == c)
    return fail(HS_E_QUBIT_RANGE, "three-qubit gate needs distinct qubits (%d, %d, %d)", a, b, c);
  auto one = [&](int kind, int q, double p0) {
    Gate v{};
    v.kind = kind;
    v.q0 = q;
    v.q1 = -1;
    v.p[0] = p0;
    out->push_back(v);
  };
  auto cx = [&](int ctl, int tgt) {
    Gate v{};
    v.kind = HS_CX;
    v.q0 = ctl;
    v.q1 = tgt;
    out->push_back(v);
  };
  const double tdg = -M_PI / 4;
  auto ccx = [&](int x, int y, int t) {
    one(HS_H, t, 0);
    cx(y, t);
    one(HS_P, t, tdg);
    cx(x, t);
    one(HS_T, t, 0);
    cx(y, t);
    one(HS_P, t, tdg);
    cx(x, t);
    one(HS_T, y, 0);
    one(HS_T, t, 0);
    one(HS_H, t, 0);
    cx(x, y);
    one(HS_T, x, 0);
    one(HS_P, y, tdg);
    cx(x, y);
  };
  if (g.kind == HS_CCX) {
    ccx(a, b, c);
  } else {
    cx(c, b);
    ccx(a, b, c);
    cx(c, b);
  }
  return HS_OK;
}

void gate_matrix(const Gate& g, cd u[4]) {
  const cd I(0.0, 1.0);
  const double th = g.p[0];
  switch (g.kind) {
    case HS_H: {
      const double r = 1.0 / sqrt(2.0);
      u[0] = r; u[1] = r; u[2] = r; u[3] = -r;
      return;
    }
    case HS_X: u[0] = 0; u[1] = 1; u[2] = 1; u[3] = 0; return;
    case HS_Y: u[0] = 0; u[1] = -I; u[2] = I; u[3] = 0; return;
    case HS_Z: u[0] = 1; u[1] = 0; u[2] = 0; u[3] = -1; return;
    case HS_S: u[0] = 1; u[1] = 0; u[2] = 0; u[3] = I; return;
    case HS_T: u[0] = 1; u[1] = 0; u[2] = 0; u[3] = std::polar(1.0, M_PI / 4); return;
    case HS_RX: {
      const double c = cos(th / 2), s = sin(th / 2);
      u[0] = c; u[1] = -I * s; u[2] = -I * s; u[3] = c;
      return;
    }
    case HS_RY: {
      const double c = cos(th / 2), s = sin(th / 2);
      u[0] = c; u[1] = -s; u[2] = s; u[3] = c;
      return;
    }
    case HS_RZ:
      u[0] = std::polar(1.0, -th / 2); u[1] = 0; u[2] = 0; u[3] = std::polar(1.0, th / 2);
      return;
    case HS_P: u[0] = 1; u[1] = 0; u[2] = 0; u[3] = std::polar(1.0, th); return;
    case HS_U3: {
      const double c = cos(th / 2), s = sin(th / 2);
      const double phi = g.p[1], lam = g.p[2];
      u[0] = c;
      u[1] = -std::polar(1.0, lam) * s;
      u[2] = std::polar(1.0, phi) * s;
      u[3] = std::polar(1.0, phi + lam) * c;
      return;
    }
    default:
      u[0] = 1; u[1] = 0; u[2] = 0; u[3] = 1;
      return;
  }
}

}  // namespace hisv
