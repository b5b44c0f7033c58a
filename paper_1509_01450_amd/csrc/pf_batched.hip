// pf_batched.hip -- many-disk forward map (first version: per-plan passes).
#include "pf_batched.hpp"

namespace pf {

template <typename T>
static int one(const Plan &p, const void *sigma, void *fr, void *fp, hipStream_t st) {
    using C = cx<T>;
    C *S = (C *)p.ws;
    C *Zr = S + (size_t)p.n_r * p.H;
    C *Zp = Zr + (size_t)p.n_r * p.H;
    int rc = launch_rows_r2c<T>(p, (const T *)sigma, nullptr, 1, p.n_r, S, nullptr,
                                (const C *)p.twN, p.sched.rows, st);
    if (rc) return rc;
    rc = launch_cols_fwd<T>(p, S, Zr, Zp, (const C *)p.spec, (const C *)p.twL, p.sched.cols, st);
    if (rc) return rc;
    return launch_rows_c2r<T>(p, Zr, Zp, 2, p.n_r, (T *)fr, (T *)fp, (const C *)p.twN,
                              p.sched.rows, st);
}

int batched_forces(const std::vector<const Plan *> &plans, const void *const *sigma,
                   void *const *f_r, void *const *f_phi, hipStream_t st) {
    for (size_t k = 0; k < plans.size(); ++k) {
        const Plan &p = *plans[k];
        int rc = p.opts.dtype == PF_F64 ? one<double>(p, sigma[k], f_r[k], f_phi[k], st)
                                        : one<float>(p, sigma[k], f_r[k], f_phi[k], st);
        if (rc) return rc;
    }
    return PF_OK;
}

void batched_forget(int64_t) {}
void autotune_plan(Plan &, hipStream_t) {}

}  // namespace pf
