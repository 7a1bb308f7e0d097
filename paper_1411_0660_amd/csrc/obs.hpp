// obs.hpp -- device workspace and launchers of the eigenvector observables.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "common.hpp"

namespace mbl {

// Column layout of ObsWork::vector_sums output (9 doubles per vector):
// 0 |psi|^2, 1 S_1, 2 sum p^2, 3 <S^z_A>, 4 <(S^z_A)^2>, 5 Re<M>, 6 Im<M>,
// 7 <M^dag M>, 8 KL(psi_v || psi_{v+1}).
constexpr int OBS_NQ = 9;

class ObsWork {
  public:
    void prepare(int L, const uint32_t *basis, int64_t dim, int nvec_max, Budget *bud,
                 hipStream_t s);
    void vector_sums(const uint32_t *basis, const double *psi, int64_t ld, int nvec,
                     double *out_dev, hipStream_t s);
    // norms2: |psi_v|^2 on the device (column 0 of vector_sums output, stride OBS_NQ);
    void entanglement(const double *psi, int64_t ldpsi, int nvec, const double *norms2,
                      double *se_dev, hipStream_t s);
    void gap_ratios(int nev, const double *E_dev, double *r_dev, hipStream_t s);
    const double *norms_dev() const { return d_out.ptr<double>() + OBS_NQ * nvmax; }
    // frees every buffer; the next prepare allocates again
    void release();

  private:
    int L = -1, nvmax = 0;
    int64_t dim = 0, gkl_stride_ = 0;     // bidiagonalisation scratch per vector (doubles)
    DevBuf d_dst, d_M, d_gkl, d_part, d_out;
};

// r, S_1 and S_E of nev vectors (device in, device out) with no device
// allocation: work in the library's fixed per-device array (mbl.h,
// mbl_observables_noalloc).
void observables_noalloc(int L, int nev, const double *evals_dev, const double *psi_dev,
                         int64_t ld, double *r_dev, double *s1_dev, double *se_dev,
                         hipStream_t s);

}  // namespace mbl
