// rates.hip -- per-SNR summaries of the library's results, host arithmetic on
// host arrays: normalised GMI, BER / SER / Q-factor from hard-decision error
// counts, hard-decision FEC pass/fail and the net rate (include/air.h), and
// the auxiliary-channel chain estimate -> rates -> NGMI.
//
// The paper judges each format by its Q-factor (from the BER) against the
// thresholds of two hard-decision FEC codes, of 6.7 % and 20 % overhead, and
// plots net throughput against distance (Section III); it prints neither the
// threshold BERs nor a net-rate formula, so the thresholds are the caller's
// and the readings below are stated in the header.
#include "../../include/air.h"
#include "host_state.h"

#include <cmath>
#include <cstdint>

using namespace air;

extern "C" {

air_status air_ngmi(const double* stats_host, int S, int m, double* ngmi_host) {
  if (!stats_host || !ngmi_host || S < 1 || m < 1) return AIR_E_INVAL;
  // H(X) = m bits under the uniform prior over M = 2^m points, so
  // 1 - (H(X) - GMI) / m = GMI / m; the standard error scales the same way
  const double inv_m = 1.0 / (double)m;
  for (int s = 0; s < S; ++s) {
    ngmi_host[2 * s] = stats_host[4 * s + 1] * inv_m;
    ngmi_host[2 * s + 1] = stats_host[4 * s + 3] * inv_m;
  }
  return AIR_OK;
}

air_status air_hd_rates(const uint64_t* counts_host, int S, int64_t N, int m, double* rates_host) {
  if (!counts_host || !rates_host || S < 1 || N < 1 || m < 1) return AIR_E_INVAL;
  const double n = (double)N;
  const double nbits = n * (double)m;
  for (int s = 0; s < S; ++s) {
    const double ber = (double)counts_host[2 * s + 1] / nbits;
    rates_host[3 * s] = ber;
    rates_host[3 * s + 1] = (double)counts_host[2 * s] / n;
    rates_host[3 * s + 2] = air_q_factor_db(ber);
  }
  return AIR_OK;
}

air_status air_fec_net(const double* ber_host, int64_t stride, int S, int m, const double* overhead,
                       const double* threshold, int F, double symbol_rate, int32_t* pass_host,
                       double* net_host, int32_t* code_host) {
  if (!ber_host || stride < 1 || S < 1 || m < 1 || !overhead || !threshold || F < 1) return AIR_E_INVAL;
  if (!(symbol_rate >= 0.0) || std::isinf(symbol_rate)) return AIR_E_INVAL;
  for (int f = 0; f < F; ++f)
    if (!(overhead[f] >= 0.0) || std::isinf(overhead[f]) || !(threshold[f] >= 0.0)) return AIR_E_INVAL;
  for (int s = 0; s < S; ++s) {
    const double ber = ber_host[(int64_t)s * stride];
    // information bits per symbol of the best code met: a code of overhead
    // OH has rate 1 / (1 + OH); a NaN BER compares false and meets none
    double best = 0.0;
    int32_t which = -1;
    for (int f = 0; f < F; ++f) {
      const bool met = ber <= threshold[f];
      if (pass_host) pass_host[(int64_t)s * F + f] = met ? 1 : 0;
      const double info = (double)m / (1.0 + overhead[f]);
      if (met && info > best) {   // strictly larger: ties keep the earlier code
        best = info;
        which = f;
      }
    }
    if (net_host) net_host[s] = best * symbol_rate;
    if (code_host) code_host[s] = which;
  }
  return AIR_OK;
}

}  // extern "C"
