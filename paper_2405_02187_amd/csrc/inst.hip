// One engine instantiation; the build compiles this file once per entry of
// XS_COMBOS with -DXS_T=<float|double> -DXS_D=<D> -DXS_Q=<Q> -DXS_NAME=<tag>.
#include "engine.hpp"

#define XS_CAT2(a, b) a##b
#define XS_CAT(a, b) XS_CAT2(a, b)

namespace xs {
EngineBase* XS_CAT(make_, XS_NAME)(xslam_ctx_s* ctx, const double T0[16], int* rc) {
  return make_engine<XS_T, XS_D, XS_Q>(ctx, T0, rc);
}
size_t XS_CAT(bytes_, XS_NAME)(const xslam_config& c, int ndd, bool wtan) {
  return engine_bytes<XS_T, XS_D, XS_Q>(c, ndd, wtan);
}
}  // namespace xs
