// Host check of the per-sample status logic the kernels share (bit tests for NaN and infinity,
// and the SF_SAMPLE_* bits from the input flag, the output flag and the final residual).
// Built and run by tests/test_abi_cpu.py; prints the number of failed checks.
#include "sf_internal.h"

#include <cstdio>
#include <cstdint>
#include <limits>

int main() {
  using sf::nonfinite_bits;
  using sf::sample_status;
  int fails = 0;
  auto chk = [&](bool c, const char* what) {
    if (!c) {
      std::printf("FAIL %s\n", what);
      ++fails;
    }
  };
  // run-time values built from their bit patterns, as the kernels see them (a NaN constant in the
  // source is folded away under no-NaN semantics, which the MFMA kernels' flags select)
  volatile uint32_t bits32[3] = {0x7f800000u, 0x7fc00000u, 0x7f800001u};   // inf, quiet NaN, signalling NaN
  volatile uint64_t bits64[2] = {0x7ff0000000000000ull, 0x7ff8000000000000ull};
  const float fi = __builtin_bit_cast(float, (uint32_t)bits32[0]);
  const float fq = __builtin_bit_cast(float, (uint32_t)bits32[1]);
  const float fs = __builtin_bit_cast(float, (uint32_t)bits32[2]);
  const double di = __builtin_bit_cast(double, (uint64_t)bits64[0]);
  const double dq = __builtin_bit_cast(double, (uint64_t)bits64[1]);
  chk(nonfinite_bits(fi) && nonfinite_bits(-fi) && nonfinite_bits(fq) && nonfinite_bits(-fq) && nonfinite_bits(fs),
      "float: infinities and NaNs are non-finite");
  chk(!nonfinite_bits(std::numeric_limits<float>::max()) && !nonfinite_bits(-std::numeric_limits<float>::max()) &&
          !nonfinite_bits(0.0f) && !nonfinite_bits(-0.0f) && !nonfinite_bits(std::numeric_limits<float>::denorm_min()),
      "float: largest, zeros and subnormals are finite");
  chk(nonfinite_bits(di) && nonfinite_bits(-di) && nonfinite_bits(dq), "double: infinities and NaN are non-finite");
  chk(!nonfinite_bits(std::numeric_limits<double>::max()) && !nonfinite_bits(1e-310) && !nonfinite_bits(0.0),
      "double: largest, subnormal and zero are finite");
  chk(nonfinite_bits(sf::quiet_nan_f32()) && nonfinite_bits(sf::quiet_nan_f64()), "NaN from bits is non-finite");
  // input flag wins and is exclusive
  chk(sample_status<float>(true, true, 5.0f, 10) == SF_SAMPLE_NONFINITE_INPUT, "input flag alone");
  // convergence at the tolerance, judged in the kernel's precision
  chk(sample_status<float>(false, false, (float)SF_CONV_TOL, 10) == 0, "at the tolerance: converged");
  chk(sample_status<float>(false, false, 1.001e-3f, 10) == SF_SAMPLE_NOT_CONVERGED, "above: not converged");
  chk(sample_status<double>(false, false, 0.0, 10) == 0, "zero residual: converged");
  chk(sample_status<double>(false, false, 2e-3, 0) == 0, "no iteration: convergence not judged");
  // non-finite results
  chk(sample_status<float>(false, true, 0.0f, 10) == SF_SAMPLE_NONFINITE, "non-finite output");
  chk(sample_status<float>(false, false, fq, 10) == (SF_SAMPLE_NONFINITE | SF_SAMPLE_NOT_CONVERGED),
      "NaN residual: non-finite and not converged");
  chk(sample_status<double>(false, false, di, 3) == (SF_SAMPLE_NONFINITE | SF_SAMPLE_NOT_CONVERGED),
      "infinite residual: non-finite and not converged");
  std::printf("%d\n", fails);
  return fails;
}
