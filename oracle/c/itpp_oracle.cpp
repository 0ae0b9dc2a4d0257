// Plain C++ dictionary-of-strings ITPP oracle -- test infrastructure only.
//
// This is the C++ twin of oracle/itpp.py, written for speed on the host so
// that larger parity cases and the CPU baseline run in seconds.  It follows
// the same steps of Algorithm 1 of arXiv 2601.14400 in the same order and
// shares no code with the GPU library:
//   * strings are std::string over the letters I X Y Z (character j is
//     qubit j) and products use the single-qubit table XY = iZ, YZ = iX,
//     ZX = iY (Pauli algebra);
//   * a gate exp(-(theta/2) Q) leaves an anticommuting P unchanged and maps
//     a commuting P to cosh(theta) P - sinh(theta) Q P (Eq. ITPP_PropRules,
//     Appendix A), theta = alpha_k * m * dtau;
//   * contributions are accumulated in an std::unordered_map (the Pauli-basis
//     re-expansion), truncated to |c| > delta (Sec. II.B) and, above K
//     strings, to the identity plus the K-1 largest |c| with ties broken by
//     the smaller (X, Z) bit integers (K-truncation, Sec. II.C);
//   * every coefficient is then divided by the identity coefficient
//     (normalisation after every elementary gate, Sec. II.C);
//   * with a Pauli-weight cutoff set (itpp_oracle_set_max_weight, the second
//     truncation rule of Sec. II.B), strings with more non-identity letters
//     than the cutoff are dropped together with the threshold, before the
//     cap (the reading of the Python oracle).
// cosh/sinh come from the C library once per gate, so results agree bit for
// bit with the Python oracle.
//
// Single-precision form: coefficients are binary32, ch and sh are the double
// values rounded to binary32, products and sums are binary32, the threshold
// compares the widened magnitude with the double delta, normalisation divides
// in double and rounds to binary32 (the same reading as the Python oracle).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

namespace {

struct Prod {
  int k;   // power of i
  char r;  // resulting letter
};

Prod mul1(char a, char b) {
  if (a == 'I') return {0, b};
  if (b == 'I') return {0, a};
  if (a == b) return {0, 'I'};
  // cyclic X->Y->Z: a b = i c ; reversed: -i c
  if ((a == 'X' && b == 'Y')) return {1, 'Z'};
  if ((a == 'Y' && b == 'Z')) return {1, 'X'};
  if ((a == 'Z' && b == 'X')) return {1, 'Y'};
  if ((a == 'Y' && b == 'X')) return {3, 'Z'};
  if ((a == 'Z' && b == 'Y')) return {3, 'X'};
  return {3, 'Y'};  // X Z = -i Y
}

bool xbit(char a) { return a == 'X' || a == 'Y'; }
bool zbit(char a) { return a == 'Z' || a == 'Y'; }

// (X, Z) integer order, most significant qubit first.
bool canonical_less(const std::string& p, const std::string& q) {
  const int n = (int)p.size();
  for (int j = n - 1; j >= 0; --j) {
    bool a = xbit(p[j]), b = xbit(q[j]);
    if (a != b) return b;
  }
  for (int j = n - 1; j >= 0; --j) {
    bool a = zbit(p[j]), b = zbit(q[j]);
    if (a != b) return b;
  }
  return false;
}

struct Oracle {
  int n = 0;
  int f32 = 0;
  std::unordered_map<std::string, double> S;   // FP64 form
  std::unordered_map<std::string, float> S32;  // FP32 form
  std::string err;
  double term_updates = 0.0;
  long long gates = 0;
  int max_weight = 0;  // 0: no weight cutoff
  // Alternative readings of where the threshold applies, for the paper's
  // threshold-sweep counts (not Algorithm 1; only with no cap binding):
  // 1 = threshold once per Trotter step, on the normalised state after its
  //     last gate (the gates of a step only propagate and normalise);
  // 2 = threshold every contribution of Eq. ITPP_PropRules before the
  //     accumulation, then the sums as in Algorithm 1;
  // 3 = as 1, on the step's coefficients before its normalisation: a string
  //     is kept when |c| times the product of the identity coefficients its
  //     gates divided by exceeds the threshold.
  int reading = 0;
};

int pauli_weight(const std::string& P) {
  int w = 0;
  for (char a : P) w += a != 'I';
  return w;
}

template <typename T>
std::unordered_map<std::string, T>& state(Oracle* o);
template <>
std::unordered_map<std::string, double>& state<double>(Oracle* o) {
  return o->S;
}
template <>
std::unordered_map<std::string, float>& state<float>(Oracle* o) {
  return o->S32;
}

template <typename T>
int evolve_impl(Oracle* o, int n_terms, const char* strings, const double* alpha, int n_gates,
                const int* term_idx, const double* mult, double dtau, long long n_steps, double delta,
                long long K);

}  // namespace

namespace {

// One elementary gate on the map S (Algorithm 1): propagate and accumulate,
// truncate (threshold, then cap), normalise.  *bI receives the identity
// coefficient before normalisation.  Returns 0, or an error code with o->err.
template <typename T>
int one_gate(Oracle* o, std::unordered_map<std::string, T>& S, const std::string& Q, double theta, double delta,
             long long K, double* bI) {
  const int n = o->n;
  const std::string ident(n, 'I');
  const T ch = (T)std::cosh(theta);
  const T sh = (T)std::sinh(theta);
  std::vector<int> sup;
  for (int j = 0; j < n; ++j)
    if (Q[j] != 'I') sup.push_back(j);
  o->term_updates += (double)S.size();
  // propagate and accumulate
  std::unordered_map<std::string, T> out;
  out.reserve(S.size() * 2 + 16);
  for (const auto& kv : S) {
    const std::string& P = kv.first;
    const T c = kv.second;
    int anti = 0;
    for (int j : sup) {
      char a = P[j], b = Q[j];
      if (a != 'I' && a != b) ++anti;
    }
    if (anti % 2) {
      if (o->reading != 2 || (double)std::fabs(c) > delta) out[P] += c;
      continue;
    }
    std::string R = P;
    int k = 0;
    for (int j : sup) {
      Prod pr = mul1(Q[j], P[j]);  // Q on the left
      k += pr.k;
      R[j] = pr.r;
    }
    k %= 4;
    if (k % 2) {
      o->err = "commuting strings gave an imaginary phase";
      return 2;
    }
    const T sign = (k == 0) ? (T)1 : (T)-1;
    const T vs = (T)(ch * c), vb = (T)((T)(-sh * sign) * c);
    if (o->reading != 2 || (double)std::fabs(vs) > delta) out[P] += vs;
    if (o->reading != 2 || (double)std::fabs(vb) > delta) out[R] += vb;
  }
  // truncate: threshold
  std::vector<std::pair<std::string, T>> kept;
  kept.reserve(out.size());
  for (auto& kv : out)
    if ((double)std::fabs(kv.second) > delta && (o->max_weight <= 0 || pauli_weight(kv.first) <= o->max_weight))
      kept.emplace_back(kv.first, kv.second);
  // truncate: cap
  if ((long long)kept.size() > K) {
    T cI = 0;
    bool have = false;
    std::vector<std::pair<std::string, T>> others;
    others.reserve(kept.size());
    for (auto& kv : kept) {
      if (kv.first == ident) {
        cI = kv.second;
        have = true;
      } else {
        others.push_back(kv);
      }
    }
    if (!have) {
      o->err = "identity coefficient was truncated";
      return 1;
    }
    auto better = [](const std::pair<std::string, T>& a, const std::pair<std::string, T>& b) {
      T fa = std::fabs(a.second), fb = std::fabs(b.second);
      if (fa != fb) return fa > fb;
      return canonical_less(a.first, b.first);
    };
    const size_t keep = (size_t)(K - 1);
    if (keep < others.size()) {
      std::nth_element(others.begin(), others.begin() + keep, others.end(), better);
      others.resize(keep);
    }
    kept.clear();
    kept.emplace_back(ident, cI);
    for (auto& kv : others) kept.push_back(kv);
  }
  // normalise (division in double)
  double cI = 0.0;
  bool have = false;
  for (auto& kv : kept)
    if (kv.first == ident) {
      cI = (double)kv.second;
      have = true;
    }
  if (!have || !(cI > 0.0) || !std::isfinite(cI)) {
    o->err = "bad identity coefficient";
    return 1;
  }
  S.clear();
  S.reserve(kept.size() * 2);
  for (auto& kv : kept) S.emplace(kv.first, (T)((double)kv.second / cI));
  ++o->gates;
  if (bI) *bI = cI;
  return 0;
}

template <typename T>
int evolve_impl(Oracle* o, int n_terms, const char* strings, const double* alpha, int n_gates,
                const int* term_idx, const double* mult, double dtau, long long n_steps, double delta,
                long long K) {
  auto& S = state<T>(o);
  const int n = o->n;
  const std::string ident(n, 'I');
  std::vector<std::string> terms(n_terms);
  for (int k = 0; k < n_terms; ++k) terms[k] = std::string(strings + (size_t)k * n, n);
  const bool per_step = o->reading == 1 || o->reading == 3;
  for (long long step = 0; step < n_steps; ++step) {
    double growth = 1.0;  // product of the step's identity coefficients before normalisation
    for (int g = 0; g < n_gates; ++g) {
      const std::string& Q = terms[term_idx[g]];
      if (Q == ident) continue;
      const double theta = alpha[term_idx[g]] * mult[g] * dtau;
      double bI = 1.0;
      const int rc = one_gate<T>(o, S, Q, theta, per_step ? -1.0 : delta, per_step ? (long long)1 << 62 : K, &bI);
      if (rc) return rc;
      growth *= bI;
    }
    if (per_step) {
      const double scale = o->reading == 3 ? growth : 1.0;
      for (auto it = S.begin(); it != S.end();) {
        if (it->first != ident && !((double)std::fabs(it->second) * scale > delta)) it = S.erase(it);
        else ++it;
      }
      if ((long long)S.size() > K) {
        o->err = "the per-step threshold reading runs without a binding cap";
        return 3;
      }
    }
  }
  return 0;
}

// Compensated running sum (Neumaier).
struct NSum {
  double s = 0.0, c = 0.0;
  void add(double v) {
    const double t = s + v;
    if (std::fabs(s) >= std::fabs(v))
      c += (s - t) + v;
    else
      c += (v - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

// Reverse-mode derivatives of L = sum_j o_j a[P_j] with the kept sets frozen
// (the steps of the reverse-mode oracle oracle/adjoint.py, in the same
// order).  One gate with string Q and angle theta maps the normalised input a
// to u (Eq. ITPP_PropRules), keeps the set S_g and divides by b_I.  Given
// lambda' = dL/da' of its output:
//   lambda_u[P] = lambda'[P] / b_I on S_g, and at the identity
//                 additionally - (sum_R lambda'_R a'_R) / b_I;
//   a commuting P with Q P = sigma R: lambda_P = ch lambda_u[P] - sigma sh lambda_u[R],
//   dL/dtheta += a_P (sh lambda_u[P] - sigma ch lambda_u[R]);
//   an anticommuting P: lambda_P = lambda_u[P].
// The kept set of gate g is the key set of the next gate's input (of the
// final state for the last gate).
int gradients_impl(Oracle* o, int n_terms, const char* strings, const double* alpha, int n_gates,
                   const int* term_idx, const double* mult, double dtau, long long n_steps, double delta,
                   long long K, int m, const char* obs, const double* oc, double* L_out, double* dtheta,
                   long long dtheta_cap, double* dalpha, double* ddtau) {
  const int n = o->n;
  const std::string ident(n, 'I');
  std::vector<std::string> terms(n_terms);
  for (int k = 0; k < n_terms; ++k) terms[k] = std::string(strings + (size_t)k * n, n);
  // forward, recording every gate's input and identity coefficient
  std::vector<std::vector<std::pair<std::string, double>>> a_in;
  std::vector<double> bI, theta_g;
  std::vector<int> term_g;
  std::vector<double> mult_g;
  for (long long step = 0; step < n_steps; ++step) {
    for (int g = 0; g < n_gates; ++g) {
      const std::string& Q = terms[term_idx[g]];
      if (Q == ident) continue;
      const double theta = alpha[term_idx[g]] * mult[g] * dtau;
      a_in.emplace_back(o->S.begin(), o->S.end());
      double b = 0.0;
      const int rc = one_gate<double>(o, o->S, Q, theta, delta, K, &b);
      if (rc) return rc;
      bI.push_back(b);
      theta_g.push_back(theta);
      term_g.push_back(term_idx[g]);
      mult_g.push_back(mult[g]);
    }
  }
  const long long G = (long long)a_in.size();
  if (G > dtheta_cap) {
    o->err = "dtheta capacity too small";
    return 3;
  }
  // seed: lambda = dL/da of the final state
  std::unordered_map<std::string, double> lam;
  NSum Ls;
  for (int j = 0; j < m; ++j) {
    const std::string P(obs + (size_t)j * n, n);
    auto it = o->S.find(P);
    if (it == o->S.end()) continue;
    lam[P] += oc[j];
    Ls.add(oc[j] * it->second);
  }
  *L_out = Ls.value();
  NSum s0;
  for (auto& kv : lam) s0.add(kv.second * o->S.at(kv.first));
  double s = s0.value();
  for (long long g = G - 1; g >= 0; --g) {
    const std::string& Q = terms[term_g[g]];
    const double ch = std::cosh(theta_g[g]), sh = std::sinh(theta_g[g]);
    // lambda_u on the kept set
    std::unordered_map<std::string, double> lam_u;
    auto put = [&](const std::string& P) {
      auto it = lam.find(P);
      lam_u[P] = (it == lam.end() ? 0.0 : it->second) / bI[g];
    };
    if (g + 1 < G)
      for (auto& kv : a_in[g + 1]) put(kv.first);
    else
      for (auto& kv : o->S) put(kv.first);
    lam_u[ident] = lam_u[ident] - s / bI[g];
    std::vector<int> sup;
    for (int j = 0; j < n; ++j)
      if (Q[j] != 'I') sup.push_back(j);
    std::unordered_map<std::string, double> lam_in;
    lam_in.reserve(a_in[g].size() * 2);
    NSum dth, ss;
    for (auto& kv : a_in[g]) {
      const std::string& P = kv.first;
      const double aP = kv.second;
      auto itp = lam_u.find(P);
      const double lp = itp == lam_u.end() ? 0.0 : itp->second;
      int anti = 0;
      for (int j : sup)
        if (P[j] != 'I' && P[j] != Q[j]) ++anti;
      double li;
      if (anti % 2) {
        li = lp;
      } else {
        std::string R = P;
        int k = 0;
        for (int j : sup) {
          Prod pr = mul1(Q[j], P[j]);
          k += pr.k;
          R[j] = pr.r;
        }
        k %= 4;
        const double sigma = k == 0 ? 1.0 : -1.0;
        auto itr = lam_u.find(R);
        const double lr = itr == lam_u.end() ? 0.0 : itr->second;
        li = ch * lp - sigma * sh * lr;
        dth.add(aP * (sh * lp - sigma * ch * lr));
      }
      lam_in[P] = li;
      ss.add(li * aP);
    }
    dtheta[g] = dth.value();
    s = ss.value();
    lam.swap(lam_in);
  }
  // chain rule to the term weights and the step
  std::vector<NSum> da(n_terms);
  NSum dd;
  for (long long g = 0; g < G; ++g) {
    da[term_g[g]].add(mult_g[g] * dtau * dtheta[g]);
    dd.add(alpha[term_g[g]] * mult_g[g] * dtheta[g]);
  }
  for (int k = 0; k < n_terms; ++k) dalpha[k] = da[k].value();
  *ddtau = dd.value();
  return 0;
}

std::string word_string(int n, int W, const uint64_t* x, const uint64_t* z) {
  std::string s(n, 'I');
  for (int j = 0; j < n; ++j) {
    const int xb = (int)((x[j >> 6] >> (j & 63)) & 1ull);
    const int zb = (int)((z[j >> 6] >> (j & 63)) & 1ull);
    s[j] = "IXZY"[xb | (zb << 1)];
  }
  (void)W;
  return s;
}

}  // namespace

extern "C" {

void* itpp_oracle_new(int n) {
  Oracle* o = new Oracle;
  o->n = n;
  o->S.emplace(std::string(n, 'I'), 1.0);
  return o;
}

void* itpp_oracle_new32(int n) {
  Oracle* o = new Oracle;
  o->n = n;
  o->f32 = 1;
  o->S32.emplace(std::string(n, 'I'), 1.0f);
  return o;
}

void itpp_oracle_free(void* h) { delete static_cast<Oracle*>(h); }

// Threshold reading of the following runs (0: Algorithm 1; 1 and 2: see Oracle::reading).
void itpp_oracle_set_reading(void* h, int reading) { static_cast<Oracle*>(h)->reading = reading; }

// Pauli-weight cutoff for the following gates (0: none).
void itpp_oracle_set_max_weight(void* h, int max_weight) { static_cast<Oracle*>(h)->max_weight = max_weight; }

const char* itpp_oracle_error(void* h) { return static_cast<Oracle*>(h)->err.c_str(); }

// strings: n_terms * n characters, row-major.
// Returns 0 on success, 1 if the identity coefficient is lost or not positive.
int itpp_oracle_evolve(void* h, int n_terms, const char* strings, const double* alpha,
                       int n_gates, const int* term_idx, const double* mult, double dtau,
                       long long n_steps, double delta, long long K) {
  Oracle* o = static_cast<Oracle*>(h);
  if (o->f32)
    return evolve_impl<float>(o, n_terms, strings, alpha, n_gates, term_idx, mult, dtau, n_steps, delta, K);
  return evolve_impl<double>(o, n_terms, strings, alpha, n_gates, term_idx, mult, dtau, n_steps, delta, K);
}

long long itpp_oracle_size(void* h) {
  Oracle* o = static_cast<Oracle*>(h);
  return (long long)(o->f32 ? o->S32.size() : o->S.size());
}

double itpp_oracle_term_updates(void* h) { return static_cast<Oracle*>(h)->term_updates; }

// Writes the state in ascending (X, Z) order: strings (size*n chars) and coefs.
void itpp_oracle_export(void* h, char* strings_out, double* coef_out) {
  Oracle* o = static_cast<Oracle*>(h);
  std::vector<std::pair<std::string, double>> v;
  if (o->f32)
    for (const auto& kv : o->S32) v.emplace_back(kv.first, (double)kv.second);
  else
    for (const auto& kv : o->S) v.emplace_back(kv.first, kv.second);
  std::sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return canonical_less(a.first, b.first); });
  for (size_t i = 0; i < v.size(); ++i) {
    std::memcpy(strings_out + i * o->n, v[i].first.data(), o->n);
    coef_out[i] = v[i].second;
  }
}

// Replaces the state (strings: count*n chars).
void itpp_oracle_import(void* h, long long count, const char* strings, const double* coef) {
  Oracle* o = static_cast<Oracle*>(h);
  o->S.clear();
  o->S32.clear();
  for (long long i = 0; i < count; ++i) {
    std::string k(strings + i * o->n, o->n);
    if (o->f32)
      o->S32[k] = (float)coef[i];
    else
      o->S[k] = coef[i];
  }
}

// Reverse-mode derivatives from the current state (see gradients_impl).
// dtheta receives one value per non-identity gate (capacity dtheta_cap),
// dalpha one per term; the state becomes the final state of the forward run.
int itpp_oracle_gradients(void* h, int n_terms, const char* strings, const double* alpha, int n_gates,
                          const int* term_idx, const double* mult, double dtau, long long n_steps, double delta,
                          long long K, int m, const char* obs, const double* oc, double* L, double* dtheta,
                          long long dtheta_cap, double* dalpha, double* ddtau) {
  Oracle* o = static_cast<Oracle*>(h);
  if (o->f32) {
    o->err = "the reverse sweep is FP64 only";
    return 3;
  }
  return gradients_impl(o, n_terms, strings, alpha, n_gates, term_idx, mult, dtau, n_steps, delta, K, m, obs, oc,
                        L, dtheta, dtheta_cap, dalpha, ddtau);
}

// Replaces the state with strings given as canonical words (W words of x
// bits, then W words of z bits per string; qubit j is bit j & 63 of word j >> 6).
void itpp_oracle_import_words(void* h, long long count, int W, const uint64_t* x, const uint64_t* z,
                              const double* coef) {
  Oracle* o = static_cast<Oracle*>(h);
  o->S.clear();
  o->S32.clear();
  for (long long i = 0; i < count; ++i) {
    std::string k = word_string(o->n, W, x + (size_t)i * W, z + (size_t)i * W);
    if (o->f32)
      o->S32[k] = (float)coef[i];
    else
      o->S[k] = coef[i];
  }
}

// Writes the state as canonical words in ascending (X, Z) order.
void itpp_oracle_export_words(void* h, int W, uint64_t* x, uint64_t* z, double* coef) {
  Oracle* o = static_cast<Oracle*>(h);
  std::vector<std::pair<std::string, double>> v;
  if (o->f32)
    for (const auto& kv : o->S32) v.emplace_back(kv.first, (double)kv.second);
  else
    for (const auto& kv : o->S) v.emplace_back(kv.first, kv.second);
  std::sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return canonical_less(a.first, b.first); });
  for (size_t i = 0; i < v.size(); ++i) {
    for (int q = 0; q < W; ++q) {
      x[i * W + q] = 0;
      z[i * W + q] = 0;
    }
    for (int j = 0; j < o->n; ++j) {
      const char a = v[i].first[j];
      if (xbit(a)) x[i * W + (j >> 6)] |= 1ull << (j & 63);
      if (zbit(a)) z[i * W + (j >> 6)] |= 1ull << (j & 63);
    }
    coef[i] = v[i].second;
  }
}

}  // extern "C"
