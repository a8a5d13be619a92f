// Extended Krylov variant (Section 4).
#include "solver.hpp"

namespace lyap {

template <typename T>
lyap_status solve_ext(const lyap_op*, const double*, int, int64_t, const lyap_opts&, lyap_result*) {
  LYAP_REQUIRE(false, LYAP_E_UNSUPPORTED, "extended Krylov not built yet");
  return LYAP_E_UNSUPPORTED;
}

template lyap_status solve_ext<float>(const lyap_op*, const double*, int, int64_t, const lyap_opts&, lyap_result*);
template lyap_status solve_ext<double>(const lyap_op*, const double*, int, int64_t, const lyap_opts&, lyap_result*);

}  // namespace lyap

extern "C" lyap_status sylv_solve(const lyap_op*, const lyap_op*, const double*, int64_t, const double*, int64_t,
                                  int32_t, const lyap_opts*, sylv_result* out) {
  lyap::set_error("sylv_solve not built yet");
  if (out) out->status = LYAP_E_UNSUPPORTED;
  return LYAP_E_UNSUPPORTED;
}

extern "C" void sylv_result_free(sylv_result* r) {
  if (!r) return;
  std::free(r->hist_m);
  std::free(r->hist_res);
  std::memset(r, 0, sizeof(*r));
}
