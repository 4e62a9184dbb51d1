// Circuit front-end (host): the QuDiet QASM reader (Sec. 4), Moment packing (Sec. 3.5), the
// decomposition of a multi-controlled X into generalized CNOTs through an intermediate level
// (Sec. 3.4), and running a circuit on a state through qd_apply_gate.
//
// QASM: ".qudit n", one "qudit NAME (d)" per qudit, the gates between ".begin" and ".end":
// "X q [a]", "H q", "Z q", "CX c t [a]" and the extension "MCT c1 .. ck t [a]". Controls fire on
// d_c - 1 (Sec. 2.1). Names are case-insensitive; '#' starts a comment.
//
// Moments: a pushed gate slides back while every qudit it touches (target and controls) holds an
// identity in the preceding Moment, so its Moment is one past the latest Moment of the earlier
// gates that share a qudit with it.
//
// Chain decomposition of X^{+a} on t controlled by c_1..c_k (values v_1..v_k): for i = 2..k,
// c_{i-1} at its marker raises c_i by 1 (c_i reaches the marker v_i + 1 exactly when c_1..c_i all
// hold their values; the marker of c_1 is v_1); c_k at its marker shifts t by a; then the chain is
// undone from i = k down to 2 with shifts d_{c_i} - 1. For two controls on (qubit, qutrit, qubit)
// this is the sequence of Sec. 3.4.
#include <algorithm>
#include <cctype>
#include <cstring>
#include <sstream>
#include <string>
#include <vector>

#include "qd_internal.h"

struct qd_circuit {
  std::vector<int32_t> dims;
  std::vector<std::string> names;
  struct G {
    int32_t kind, target, a;
    std::vector<int32_t> ctl, cval;
  };
  std::vector<G> gates;
};

namespace qd {
namespace {

int check_add(const qd_circuit* c, int32_t kind, int32_t target, int32_t a, const int32_t* controls,
              const int32_t* values, int32_t m) {
  const int n = int(c->dims.size());
  if (kind != QD_GATE_X && kind != QD_GATE_Z && kind != QD_GATE_F) return fail(QD_EINVAL, "gate kind must be X, Z or F");
  if (target < 0 || target >= n) return fail(QD_EINVAL, "target outside the register");
  if (kind == QD_GATE_X && (a < 1 || a > c->dims[size_t(target)] - 1)) return fail(QD_EINVAL, "shift outside 1..d-1");
  if (m < 0 || m >= n) return fail(QD_EINVAL, "bad control count");
  if (m && (!controls || !values)) return fail(QD_EINVAL, "null controls");
  std::vector<bool> seen(size_t(n), false);
  seen[size_t(target)] = true;
  for (int j = 0; j < m; ++j) {
    if (controls[j] < 0 || controls[j] >= n || seen[size_t(controls[j])]) return fail(QD_EINVAL, "bad or repeated control");
    seen[size_t(controls[j])] = true;
    if (values[j] < 0 || values[j] >= c->dims[size_t(controls[j])]) return fail(QD_EINVAL, "control value outside 0..d-1");
  }
  return QD_OK;
}

void add_gate(qd_circuit* c, int32_t kind, int32_t target, int32_t a, const int32_t* controls, const int32_t* values,
              int32_t m) {
  qd_circuit::G g;
  g.kind = kind;
  g.target = target;
  g.a = kind == QD_GATE_X ? a : 0;
  g.ctl.assign(controls, controls + m);
  g.cval.assign(values, values + m);
  c->gates.push_back(std::move(g));
}

std::string lower(std::string s) {
  for (char& ch : s) ch = char(std::tolower(static_cast<unsigned char>(ch)));
  return s;
}

bool all_digits(const std::string& s) {
  return !s.empty() && std::all_of(s.begin(), s.end(), [](char ch) { return std::isdigit(static_cast<unsigned char>(ch)); });
}

int line_fail(int lineno, const std::string& what) {
  return fail(QD_EINVAL, "qasm line " + std::to_string(lineno) + ": " + what);
}

int parse(const char* text, qd_circuit* c) {
  std::istringstream in(text);
  std::string raw;
  int lineno = 0, declared = -1;
  enum { HEAD, BODY, DONE } st = HEAD;
  while (std::getline(in, raw)) {
    ++lineno;
    const size_t hash = raw.find('#');
    if (hash != std::string::npos) raw.resize(hash);
    std::string spaced;
    for (char ch : raw) {
      if (ch == '(' || ch == ')') {
        spaced += ' ';
        spaced += ch;
        spaced += ' ';
      } else {
        spaced += ch;
      }
    }
    std::istringstream ls(spaced);
    std::vector<std::string> tok;
    for (std::string t; ls >> t;) tok.push_back(t);
    if (tok.empty()) continue;
    const std::string key = lower(tok[0]);
    if (st == HEAD) {
      if (key == ".qudit") {
        if (tok.size() != 2 || !all_digits(tok[1]) || declared >= 0) return line_fail(lineno, "bad .qudit");
        declared = std::stoi(tok[1]);
      } else if (key == "qudit") {
        if (tok.size() != 5 || tok[2] != "(" || tok[4] != ")" || !all_digits(tok[3]) || tok[3].size() > 4)
          return line_fail(lineno, "bad qudit declaration");
        const std::string name = lower(tok[1]);
        const int d = std::stoi(tok[3]);
        if (std::find(c->names.begin(), c->names.end(), name) != c->names.end() || d < 2 || d > QD_MAX_RADIX ||
            int(c->names.size()) >= QD_MAX_QUDITS)
          return line_fail(lineno, "duplicate qudit, dimension outside 2..256 or too many qudits");
        c->names.push_back(name);
        c->dims.push_back(d);
      } else if (key == ".begin") {
        if (c->names.empty() || (declared >= 0 && declared != int(c->names.size())))
          return line_fail(lineno, "qudit count does not match .qudit");
        st = BODY;
      } else {
        return line_fail(lineno, "unexpected line before .begin");
      }
      continue;
    }
    if (st == DONE) return line_fail(lineno, "text after .end");
    if (key == ".end") {
      st = DONE;
      continue;
    }
    std::vector<std::string> args(tok.begin() + 1, tok.end());
    int shift = 0;
    bool has_shift = false;
    if (!args.empty()) {
      const std::string& last = args.back();
      const std::string body = (!last.empty() && last[0] == '-') ? last.substr(1) : last;
      if (all_digits(body) && body.size() <= 6) {
        shift = std::stoi(last);
        has_shift = true;
        args.pop_back();
      }
    }
    std::vector<int32_t> wires;
    for (const std::string& a : args) {
      const auto it = std::find(c->names.begin(), c->names.end(), lower(a));
      if (it == c->names.end()) return line_fail(lineno, "unknown qudit " + a);
      wires.push_back(int32_t(it - c->names.begin()));
    }
    std::vector<int32_t> sorted = wires;
    std::sort(sorted.begin(), sorted.end());
    const bool distinct = std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end();
    if (key == "x" || key == "h" || key == "z") {
      if (wires.size() != 1 || (key != "x" && has_shift)) return line_fail(lineno, "bad " + tok[0] + " gate");
      const int32_t t = wires[0];
      const int32_t a = has_shift ? shift : 1;
      const int32_t kind = key == "x" ? QD_GATE_X : (key == "h" ? QD_GATE_F : QD_GATE_Z);
      if (kind == QD_GATE_X && (a < 1 || a > c->dims[size_t(t)] - 1)) return line_fail(lineno, "shift outside 1..d-1");
      add_gate(c, kind, t, a, nullptr, nullptr, 0);
    } else if (key == "cx" || key == "mct") {
      if (wires.size() < 2 || (key == "cx" && wires.size() != 2) || !distinct) return line_fail(lineno, "bad " + tok[0] + " gate");
      const int32_t t = wires.back();
      const int32_t a = has_shift ? shift : 1;
      if (a < 1 || a > c->dims[size_t(t)] - 1) return line_fail(lineno, "shift outside 1..d-1");
      std::vector<int32_t> ctl(wires.begin(), wires.end() - 1), val;
      for (int32_t q : ctl) val.push_back(c->dims[size_t(q)] - 1);
      add_gate(c, QD_GATE_X, t, a, ctl.data(), val.data(), int32_t(ctl.size()));
    } else {
      return line_fail(lineno, "unknown gate " + tok[0]);
    }
  }
  if (st != DONE) return fail(QD_EINVAL, "qasm: missing .begin or .end");
  return QD_OK;
}

}  // namespace
}  // namespace qd

using namespace qd;

extern "C" {

int qd_circuit_create(const int32_t* dims, int32_t n, qd_circuit** out) {
  if (!dims || !out || n < 1 || n > QD_MAX_QUDITS) return fail(QD_EINVAL, "bad register");
  *out = nullptr;
  for (int q = 0; q < n; ++q)
    if (dims[q] < 2 || dims[q] > QD_MAX_RADIX) return fail(QD_EDIM, "qudit dimension must be 2..256");
  qd_circuit* c = new qd_circuit;
  c->dims.assign(dims, dims + n);
  for (int q = 0; q < n; ++q) c->names.push_back("q" + std::to_string(q));
  *out = c;
  return QD_OK;
}

int qd_circuit_add(qd_circuit* c, int32_t kind, int32_t target, int32_t a, const int32_t* controls,
                   const int32_t* control_values, int32_t m) {
  if (!c) return fail(QD_EINVAL, "null circuit");
  const int rc = check_add(c, kind, target, a, controls, control_values, m);
  if (rc) return rc;
  add_gate(c, kind, target, a, controls, control_values, m);
  return QD_OK;
}

int qd_qasm_parse(const char* text, qd_circuit** out) {
  if (!text || !out) return fail(QD_EINVAL, "null argument");
  *out = nullptr;
  qd_circuit* c = new qd_circuit;
  const int rc = parse(text, c);
  if (rc) {
    delete c;
    return rc;
  }
  *out = c;
  return QD_OK;
}

int qd_circuit_size(const qd_circuit* c, int32_t* n_qudits, int64_t* n_gates) {
  if (!c) return fail(QD_EINVAL, "null circuit");
  if (n_qudits) *n_qudits = int32_t(c->dims.size());
  if (n_gates) *n_gates = int64_t(c->gates.size());
  return QD_OK;
}

int qd_circuit_dims(const qd_circuit* c, int32_t* dims_out) {
  if (!c || !dims_out) return fail(QD_EINVAL, "null argument");
  std::copy(c->dims.begin(), c->dims.end(), dims_out);
  return QD_OK;
}

int qd_circuit_name(const qd_circuit* c, int32_t q, char* buf, int32_t buflen) {
  if (!c || !buf || buflen < 1) return fail(QD_EINVAL, "null argument");
  if (q < 0 || q >= int32_t(c->names.size())) return fail(QD_EINVAL, "qudit outside the register");
  const std::string& s = c->names[size_t(q)];
  if (int32_t(s.size()) + 1 > buflen) return fail(QD_EINVAL, "buffer too small");
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return QD_OK;
}

int qd_circuit_gate(const qd_circuit* c, int64_t i, int32_t* kind, int32_t* target, int32_t* a, int32_t* m,
                    int32_t* controls, int32_t* control_values) {
  if (!c) return fail(QD_EINVAL, "null circuit");
  if (i < 0 || i >= int64_t(c->gates.size())) return fail(QD_EINVAL, "gate index outside the circuit");
  const qd_circuit::G& g = c->gates[size_t(i)];
  if (kind) *kind = g.kind;
  if (target) *target = g.target;
  if (a) *a = g.a;
  if (m) *m = int32_t(g.ctl.size());
  if (controls) std::copy(g.ctl.begin(), g.ctl.end(), controls);
  if (control_values) std::copy(g.cval.begin(), g.cval.end(), control_values);
  return QD_OK;
}

int qd_circuit_moments(const qd_circuit* c, int32_t* moment_out, int32_t* depth) {
  if (!c) return fail(QD_EINVAL, "null circuit");
  std::vector<int32_t> last(c->dims.size(), -1);
  int32_t deepest = -1;
  for (size_t i = 0; i < c->gates.size(); ++i) {
    const qd_circuit::G& g = c->gates[i];
    int32_t m = last[size_t(g.target)];
    for (int32_t q : g.ctl) m = std::max(m, last[size_t(q)]);
    ++m;
    last[size_t(g.target)] = m;
    for (int32_t q : g.ctl) last[size_t(q)] = m;
    if (moment_out) moment_out[i] = m;
    deepest = std::max(deepest, m);
  }
  if (depth) *depth = deepest + 1;
  return QD_OK;
}

int qd_circuit_decompose(const qd_circuit* c, qd_circuit** out) {
  if (!c || !out) return fail(QD_EINVAL, "null argument");
  *out = nullptr;
  // every multi-controlled X needs a free level above each chained control's value
  for (const qd_circuit::G& g : c->gates)
    if (g.kind == QD_GATE_X && g.ctl.size() >= 2)
      for (size_t i = 1; i < g.ctl.size(); ++i)
        if (g.cval[i] + 2 > c->dims[size_t(g.ctl[i])])
          return fail(QD_EDIM, "control qudit " + std::to_string(g.ctl[i]) + " has no free level for the chain marker");
  qd_circuit* o = new qd_circuit;
  o->dims = c->dims;
  o->names = c->names;
  for (const qd_circuit::G& g : c->gates) {
    const size_t k = g.ctl.size();
    if (g.kind != QD_GATE_X || k < 2) {
      o->gates.push_back(g);
      continue;
    }
    std::vector<int32_t> marker(k);
    marker[0] = g.cval[0];
    for (size_t i = 1; i < k; ++i) marker[i] = g.cval[i] + 1;
    for (size_t i = 1; i < k; ++i) add_gate(o, QD_GATE_X, g.ctl[i], 1, &g.ctl[i - 1], &marker[i - 1], 1);
    add_gate(o, QD_GATE_X, g.target, g.a, &g.ctl[k - 1], &marker[k - 1], 1);
    for (size_t i = k - 1; i >= 1; --i)
      add_gate(o, QD_GATE_X, g.ctl[i], c->dims[size_t(g.ctl[i])] - 1, &g.ctl[i - 1], &marker[i - 1], 1);
  }
  *out = o;
  return QD_OK;
}

int qd_circuit_apply(qd_state* s, const qd_circuit* c) {
  if (!s || !c) return fail(QD_EINVAL, "null argument");
  // gates were checked against the circuit's register when added, so with equal registers every
  // qd_apply_gate below passes validation
  const std::vector<int32_t> sd(s->reg.dims, s->reg.dims + s->reg.n);
  if (sd != c->dims) return fail(QD_EDIM, "circuit register differs from the state's");
  std::vector<double> U;
  for (const qd_circuit::G& g : c->gates) {
    const int d = c->dims[size_t(g.target)];
    U.assign(2 * size_t(d) * size_t(d), 0.0);
    int rc = qd_gate_matrix(g.kind, d, g.kind == QD_GATE_X ? g.a : 0, U.data());
    if (rc) return rc;
    rc = qd_apply_gate(s, &g.target, 1, g.ctl.data(), g.cval.data(), int32_t(g.ctl.size()), U.data());
    if (rc) return rc;
  }
  return QD_OK;
}

int qd_circuit_apply_sparse(qd_sparse* s, const qd_circuit* c) {
  if (!s || !c) return fail(QD_EINVAL, "null argument");
  const Register& r = sparse_register(s);
  const std::vector<int32_t> sd(r.dims, r.dims + r.n);
  if (sd != c->dims) return fail(QD_EDIM, "circuit register differs from the state's");
  std::vector<SparseGate> seq(c->gates.size());
  for (size_t i = 0; i < c->gates.size(); ++i) {
    const qd_circuit::G& g = c->gates[i];
    const int d = c->dims[size_t(g.target)];
    SparseGate& q = seq[i];
    q.t = {g.target};
    q.c = g.ctl;
    q.v = g.cval;
    q.U.assign(2 * size_t(d) * size_t(d), 0.0);
    int rc = qd_gate_matrix(g.kind, d, g.kind == QD_GATE_X ? g.a : 0, q.U.data());
    if (rc) return rc;
  }
  return sparse_apply_gates(s, seq.data(), seq.size(), 0);
}

void qd_circuit_free(qd_circuit* c) { delete c; }

}  // extern "C"
