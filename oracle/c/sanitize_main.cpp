// Driver for a sanitizer build of the C++ oracle (test infrastructure only):
// built with -fsanitize=address,undefined together with itpp_oracle.cpp by
// tests/test_c_oracle.py, it runs every entry point on a small capped TFIM
// chain (both precisions, the weight cutoff, the threshold readings, word
// import/export and the reverse sweep) and exits non-zero on any failure.
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

extern "C" {
void* itpp_oracle_new(int n);
void* itpp_oracle_new32(int n);
void itpp_oracle_free(void* h);
void itpp_oracle_set_reading(void* h, int reading);
void itpp_oracle_set_max_weight(void* h, int max_weight);
int itpp_oracle_evolve(void* h, int n_terms, const char* strings, const double* alpha, int n_gates,
                       const int* term_idx, const double* mult, double dtau, long long n_steps, double delta,
                       long long K);
long long itpp_oracle_size(void* h);
void itpp_oracle_export(void* h, char* strings_out, double* coef_out);
void itpp_oracle_import(void* h, long long count, const char* strings, const double* coef);
void itpp_oracle_import_words(void* h, long long count, int W, const uint64_t* x, const uint64_t* z,
                              const double* coef);
void itpp_oracle_export_words(void* h, int W, uint64_t* x, uint64_t* z, double* coef);
int itpp_oracle_gradients(void* h, int n_terms, const char* strings, const double* alpha, int n_gates,
                          const int* term_idx, const double* mult, double dtau, long long n_steps, double delta,
                          long long K, int m, const char* obs, const double* oc, double* L, double* dtheta,
                          long long dtheta_cap, double* dalpha, double* ddtau);
}

int main() {
  const int n = 10;
  // open TFIM: ZZ bonds then X sites, first order
  std::vector<std::string> terms;
  std::vector<double> alpha;
  for (int i = 0; i + 1 < n; ++i) {
    std::string s(n, 'I');
    s[i] = s[i + 1] = 'Z';
    terms.push_back(s);
    alpha.push_back(-1.0);
  }
  for (int i = 0; i < n; ++i) {
    std::string s(n, 'I');
    s[i] = 'X';
    terms.push_back(s);
    alpha.push_back(-0.9);
  }
  std::string flat;
  for (auto& t : terms) flat += t;
  const int G = (int)terms.size();
  std::vector<int> idx(G);
  std::vector<double> mult(G, 1.0);
  for (int g = 0; g < G; ++g) idx[g] = g;
  int fails = 0;
  for (int prec = 0; prec < 2; ++prec)
    for (int wmax : {0, 3})
      for (int reading : {0, 1, 2}) {
        if (prec == 1 && reading != 0) continue;
        void* h = prec ? itpp_oracle_new32(n) : itpp_oracle_new(n);
        itpp_oracle_set_max_weight(h, wmax);
        itpp_oracle_set_reading(h, reading);
        const long long K = reading == 1 ? (1LL << 40) : 150;
        if (itpp_oracle_evolve(h, G, flat.c_str(), alpha.data(), G, idx.data(), mult.data(), 0.05, 4, 1e-8, K)) ++fails;
        const long long cnt = itpp_oracle_size(h);
        std::vector<char> s((size_t)cnt * n);
        std::vector<double> c((size_t)cnt);
        itpp_oracle_export(h, s.data(), c.data());
        itpp_oracle_import(h, cnt, s.data(), c.data());
        if (itpp_oracle_size(h) != cnt) ++fails;
        itpp_oracle_free(h);
      }
  // word import / export and the reverse sweep
  void* h = itpp_oracle_new(n);
  std::vector<uint64_t> x = {0, 1, 6}, z = {0, 2, 6};
  std::vector<double> c = {1.0, 0.25, -0.5};
  itpp_oracle_import_words(h, 3, 1, x.data(), z.data(), c.data());
  std::vector<uint64_t> xo(3), zo(3);
  std::vector<double> co(3);
  itpp_oracle_export_words(h, 1, xo.data(), zo.data(), co.data());
  itpp_oracle_free(h);
  h = itpp_oracle_new(n);
  double L = 0.0, dd = 0.0;
  std::vector<double> dth(8 * G), da(G);
  if (itpp_oracle_gradients(h, G, flat.c_str(), alpha.data(), G, idx.data(), mult.data(), 0.05, 3, 1e-8, 200, G,
                            flat.c_str(), alpha.data(), &L, dth.data(), (long long)dth.size(), da.data(), &dd))
    ++fails;
  itpp_oracle_free(h);
  std::printf("sanitized oracle run: %d failures, L = %.12f\n", fails, L);
  return fails ? 1 : 0;
}
