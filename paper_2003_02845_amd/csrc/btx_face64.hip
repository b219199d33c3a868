// Face-kernel instances in double (see btx_dev.h).
#include "btx_dev.h"

namespace {
using btx::FaceShape;
template <typename T, int NCH, int MAXT, bool SPLIT>
const void *face_fn_t(int ce)
{
  if constexpr (NCH == 8) {
    switch (ce) {
    case 3: return (const void *)face_kernel<T, 8, 3, MAXT, SPLIT>;
    case 4: return (const void *)face_kernel<T, 8, 4, MAXT, SPLIT>;
    case 5: return (const void *)face_kernel<T, 8, 5, MAXT, SPLIT>;
    case 6: return (const void *)face_kernel<T, 8, 6, MAXT, SPLIT>;
    case 8: return (const void *)face_kernel<T, 8, 8, MAXT, SPLIT>;
    default: return nullptr;
    }
  } else {
    switch (ce) {
    case 4: return (const void *)face_kernel<T, 4, 4, MAXT, SPLIT>;
    case 5: return (const void *)face_kernel<T, 4, 5, MAXT, SPLIT>;
    case 6: return (const void *)face_kernel<T, 4, 6, MAXT, SPLIT>;
    case 7: return (const void *)face_kernel<T, 4, 7, MAXT, SPLIT>;
    case 8: return (const void *)face_kernel<T, 4, 8, MAXT, SPLIT>;
    case 12: return (const void *)face_kernel<T, 4, 12, MAXT, SPLIT>;
    case 16: return (const void *)face_kernel<T, 4, 16, MAXT, SPLIT>;
    default: return nullptr;
    }
  }
}

template <typename T, int NCH>
const void *face_fn_g(int ce)
{
  switch (ce) {
  case 4: return (const void *)face_kernel<T, NCH, 4, 1024, false, true>;
  case 8: return (const void *)face_kernel<T, NCH, 8, 1024, false, true>;
  case 16: return (const void *)face_kernel<T, NCH, 16, 1024, false, true>;
  default: return nullptr;
  }
}

// the face-kernel instance of a shape
template <typename T>
const void *face_fn(const FaceShape &f)
{
  if (f.ce == 0) return nullptr;
  if (f.gtab) {
    if (f.split) return nullptr;
    return f.nch == 4 ? face_fn_g<T, 4>(f.ce) : f.nch == 2 ? face_fn_g<T, 2>(f.ce)
                      : f.nch == 1 ? face_fn_g<T, 1>(f.ce) : nullptr;
  }
  if (f.nch == 4) return f.split ? face_fn_t<T, 4, 512, true>(f.ce) : face_fn_t<T, 4, 512, false>(f.ce);
  if (f.maxt == 768) return f.split ? face_fn_t<T, 8, 768, true>(f.ce) : face_fn_t<T, 8, 768, false>(f.ce);
  if constexpr (sizeof(T) == 4)
    return f.split ? face_fn_t<T, 8, 1024, true>(f.ce) : face_fn_t<T, 8, 1024, false>(f.ce);
  return nullptr;
}

}  // namespace

const void *btx::face_fn_f64(const FaceShape &f) { return face_fn<double>(f); }
