// Per-column steps shared by the dense strip passes (strip.hip) and the sparse column passes
// (sparse.hip). Each pass computes, for every column j of A, the dots t of a_j with its ND
// m-vectors (vec0, vec1), then derives the column's coefficients for the row accumulation (and
// column-side outputs):
//   OpMatvec: coef = d2_j t                                    (CG matvec, Alg. 1 step 3)
//   OpMatvec2: coef_k = d2_j t_k, k = 0, 1                     (A D^2 A^T [v0 v1] in one pass)
//   OpResid:  r_d = t + s_j - c_j (stored, sum of squares kept); coefs x_j and
//             sigma mu / s_j + d2_j r_d                         (residual pass, Sec. 5)
//   OpDir:    ds_j = -r_d,j - t (stored); coef = d2_j t          (direction pass, eq. ipm_inf)
// For Algorithm 2 (a.feasible) r_d is taken as 0 in the coefficient and in ds (eqns. pdef, dels).
#pragma once

#include "kernels.hpp"

namespace ipmsk {

struct OpMatvec {
    static constexpr int ND = 1, NACC = 1, NCR = 0;
    static constexpr bool PF = true;
    struct S {};
    __device__ __forceinline__ static S init(const StripCall&) { return {}; }
    __device__ __forceinline__ static double pre(const StripCall& a, int64_t j, bool valid) { return valid ? a.d2[j] : 0.0; }
    template <typename ACC>
    __device__ __forceinline__ static void column(const StripCall& a, const S&, int64_t j, bool valid, bool, const ACC* dot,
                                  ACC* coef, double*, double pf) {
        coef[0] = valid ? (ACC)pf * dot[0] : (ACC)0;
    }
};

struct OpMatvec2 {
    static constexpr int ND = 2, NACC = 2, NCR = 0;
    static constexpr bool PF = true;
    struct S {};
    __device__ __forceinline__ static S init(const StripCall&) { return {}; }
    __device__ __forceinline__ static double pre(const StripCall& a, int64_t j, bool valid) { return valid ? a.d2[j] : 0.0; }
    template <typename ACC>
    __device__ __forceinline__ static void column(const StripCall& a, const S&, int64_t j, bool valid, bool, const ACC* dot,
                                  ACC* coef, double*, double pf) {
        coef[0] = valid ? (ACC)pf * dot[0] : (ACC)0;
        coef[1] = valid ? (ACC)pf * dot[1] : (ACC)0;
    }
};

struct OpResid {
    static constexpr bool PF = false;
    __device__ __forceinline__ static double pre(const StripCall&, int64_t, bool) { return 0.0; }
    static constexpr int ND = 1, NACC = 2, NCR = 1;
    struct S { double smu; };
    __device__ __forceinline__ static S init(const StripCall& a) { return S{a.scal[SC_SMU]}; }
    template <typename ACC>
    __device__ __forceinline__ static void column(const StripCall& a, const S& st, int64_t j, bool valid, bool writer,
                                  const ACC* dot, ACC* coef, double* cr, double) {
        if (!valid) { coef[0] = coef[1] = (ACC)0; return; }
        const double sj = a.s[j];
        const double rdj = (double)dot[0] + sj - a.c[j];
        if (writer) { a.rd_out[j] = rdj; cr[0] += rdj * rdj; }
        coef[0] = (ACC)a.x[j];
        coef[1] = (ACC)(a.feasible ? st.smu / sj : st.smu / sj + a.d2[j] * rdj);
    }
};

struct OpDir {
    static constexpr bool PF = false;
    __device__ __forceinline__ static double pre(const StripCall&, int64_t, bool) { return 0.0; }
    static constexpr int ND = 1, NACC = 1, NCR = 0;
    struct S {};
    __device__ __forceinline__ static S init(const StripCall&) { return {}; }
    template <typename ACC>
    __device__ __forceinline__ static void column(const StripCall& a, const S&, int64_t j, bool valid, bool writer,
                                  const ACC* dot, ACC* coef, double*, double) {
        if (!valid) { coef[0] = (ACC)0; return; }
        const double t = (double)dot[0];
        if (writer) a.ds_out[j] = a.feasible ? -t : -a.rd[j] - t;
        coef[0] = (ACC)(a.d2[j] * t);
    }
};


}  // namespace ipmsk
