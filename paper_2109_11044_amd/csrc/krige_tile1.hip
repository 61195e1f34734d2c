// krige_tile1.hip -- launches of the mixed grid product's tiles with one
// node fragment per wave (the default tile of 128 nodes x 256 realizations
// and the tiles for calls of up to 64 and 128 realizations).  Built with
// machine sinking off: their coefficient reads, issued a block ahead of
// the conditional matrix instructions, must stay there.
#include "krige_mixed.hpp"

namespace cesim {

cesim_status launch_split3_one_fragment(int nu, int nb, bool f16, dim3 grid, hipStream_t s,
                                        float* fields, int m1, int M, int R, int Rp,
                                        const void* Bh, const void* Bl, const float* colscale,
                                        const float* yhat, int n, const float2* st,
                                        const float4* circ, float xcut, float ux, float uxy,
                                        float uyx, float uy, float dx, float dy, float kscale,
                                        const int* fail) {
  if (nb != 2 && nb != 4 && nb != 8) return CESIM_ERR_INVALID_ARG;
#define CESIM_K1(NU, NB, H)                                                                    \
  k_krige_split3<NU, 1, NB, H><<<grid, 256, 0, s>>>(                                          \
      fields, m1, M, R, Rp, static_cast<const H*>(Bh), static_cast<const H*>(Bl), colscale,    \
      yhat, n, st, circ, xcut, ux, uxy, uyx, uy, dx, dy, kscale, fail)
#define CESIM_K1_NB(NU, H)                   \
  switch (nb) {                              \
    case 2: CESIM_K1(NU, 2, H); break;       \
    case 4: CESIM_K1(NU, 4, H); break;       \
    default: CESIM_K1(NU, 8, H); break;      \
  }
#define CESIM_K1_NU(H)                       \
  switch (nu) {                              \
    case 0: CESIM_K1_NB(0, H) break;         \
    case 1: CESIM_K1_NB(1, H) break;         \
    default: CESIM_K1_NB(2, H) break;        \
  }
  if (f16) {
    CESIM_K1_NU(_Float16)
  } else {
    CESIM_K1_NU(__bf16)
  }
#undef CESIM_K1_NU
#undef CESIM_K1_NB
#undef CESIM_K1
  CESIM_HIP(hipGetLastError());
  return CESIM_OK;
}

}  // namespace cesim
