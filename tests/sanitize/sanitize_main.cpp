// sanitize_main.cpp -- TEST ONLY: runs the oracle (oracle/gwf_oracle.cpp)
// and the host build of the kernels' per-point mathematics
// (tests/model_host/model_host.hip) under AddressSanitizer and
// UndefinedBehaviorSanitizer, on a workload read from a file, and writes
// their outputs for the test to compare with the uninstrumented builds.
// Any sanitizer report ends the process with a nonzero status.
//
// usage: sanitize_main in.bin out.bin
//   in.bin:  int64 n, n_site, flags, P; double par[13][n], sites[n_site][7],
//            fmin[n]; int32 npts[n]; double gbar[P][P][n]
//   out.bin: doubles, in this order: oracle snr[n], Fisher [P][P][n],
//            strain [n_ifo][total][2], strain derivatives [P][n_ifo][total][2],
//            tangent snr2 [2][n] and Fisher [2][P][P][n] (site 0, longitude);
//            host-build snr[n], Fisher [P][P][n], adjoint [n][n_site][4];
//            Jacobi condition numbers of the oracle's matrices [n]
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
int orc_n_ifo(int n_site, const double* sites);
int orc_fisher(int64_t n, const double* par, int64_t ld, const double* tc_s, int n_site, const double* sites,
               const double* fmin, const double* fmax, const int32_t* npts, const uint8_t* active, int flags,
               int nthreads, double* snr, double* snr_ifo, double* fisher, double* fisher_ifo);
int orc_waveform(int64_t n, const double* par, int64_t ld, const double* tc_s, int n_site, const double* sites,
                 const double* fmin, const double* fmax, const int32_t* npts, int flags, int nthreads,
                 const int64_t* offsets, int64_t total, double* h);
int orc_waveform_deriv(int64_t n, const double* par, int64_t ld, const double* tc_s, int n_site,
                       const double* sites, const double* fmin, const double* fmax, const int32_t* npts,
                       int flags, int nthreads, const int64_t* offsets, int64_t total, double* dh);
int orc_fisher_tangent(int64_t n, const double* par, int64_t ld, const double* tc_s, int n_site,
                       const double* sites, const double* fmin, const double* fmax, const int32_t* npts,
                       const uint8_t* active, int flags, int nthreads, int site, int which, double* snr2,
                       double* fisher);
int model_fisher_host(int64_t n, const double* par, int64_t ld, const double* fmin, const double* fmax,
                      const int32_t* npts, int n_site, const double* sites, uint32_t flags, double* fisher,
                      double* snr, int32_t* status);
int model_adjoint_host(int64_t n, const double* par, int64_t ld, const double* fmin, const double* fmax,
                       const int32_t* npts, int n_site, const double* sites, uint32_t flags, const double* gbar,
                       double w_snr, double w_fisher, double* grad_event);
int model_jacobi_cond_host(int P, int64_t n, const double* F, double* cond, int32_t* sweeps);
}

template <class T>
static void read(FILE* f, std::vector<T>& v, size_t count) {
  v.resize(count);
  if (count && fread(v.data(), sizeof(T), count, f) != count) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s in.bin out.bin\n", argv[0]);
    return 2;
  }
  FILE* in = fopen(argv[1], "rb");
  if (!in) return 2;
  std::vector<int64_t> hdr;
  read(in, hdr, 4);
  const int64_t n = hdr[0];
  const int n_site = (int)hdr[1], flags = (int)hdr[2], P = (int)hdr[3];
  std::vector<double> par, sites, fmin, gbar;
  std::vector<int32_t> npts;
  read(in, par, 13 * n);
  read(in, sites, 7 * (size_t)n_site);
  read(in, fmin, n);
  read(in, npts, n);
  read(in, gbar, (size_t)P * P * n);
  fclose(in);

  const int nifo = orc_n_ifo(n_site, sites.data());
  std::vector<int64_t> off(n);
  int64_t total = 0;
  for (int64_t e = 0; e < n; ++e) {
    off[e] = total;
    total += npts[e];
  }
  std::vector<double> snr(n), snr_ifo(nifo * n), F((size_t)P * P * n);
  orc_fisher(n, par.data(), n, nullptr, n_site, sites.data(), fmin.data(), nullptr, npts.data(), nullptr, flags, 1,
             snr.data(), snr_ifo.data(), F.data(), nullptr);
  std::vector<double> h((size_t)nifo * total * 2), dh((size_t)P * nifo * total * 2);
  orc_waveform(n, par.data(), n, nullptr, n_site, sites.data(), fmin.data(), nullptr, npts.data(), flags, 1,
               off.data(), total, h.data());
  orc_waveform_deriv(n, par.data(), n, nullptr, n_site, sites.data(), fmin.data(), nullptr, npts.data(), flags, 1,
                     off.data(), total, dh.data());
  std::vector<double> t_snr2(2 * n), t_F(2 * (size_t)P * P * n);
  orc_fisher_tangent(n, par.data(), n, nullptr, n_site, sites.data(), fmin.data(), nullptr, npts.data(), nullptr,
                     flags, 1, 0, 1, t_snr2.data(), t_F.data());
  std::vector<double> m_snr(n), m_F((size_t)P * P * n), m_adj((size_t)n * n_site * 4);
  std::vector<int32_t> m_st(n);
  model_fisher_host(n, par.data(), n, fmin.data(), nullptr, npts.data(), n_site, sites.data(), (uint32_t)flags,
                    m_F.data(), m_snr.data(), m_st.data());
  model_adjoint_host(n, par.data(), n, fmin.data(), nullptr, npts.data(), n_site, sites.data(), (uint32_t)flags,
                     gbar.data(), 0.7, 1.3, m_adj.data());
  std::vector<double> cond(n);
  std::vector<int32_t> sweeps(n);
  model_jacobi_cond_host(P, n, F.data(), cond.data(), sweeps.data());

  FILE* out = fopen(argv[2], "wb");
  if (!out) return 2;
  for (const std::vector<double>* v : {&snr, &F, &h, &dh, &t_snr2, &t_F, &m_snr, &m_F, &m_adj, &cond})
    fwrite(v->data(), sizeof(double), v->size(), out);
  fclose(out);
  printf("sanitized run ok: %lld events, %d interferometers, %lld points\n", (long long)n, nifo, (long long)total);
  return 0;
}
