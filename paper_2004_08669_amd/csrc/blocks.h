// GEMM operand accessors and epilogues for the spin-major block layout of the
// CTMRG matrices: every (q m) x (q m) matrix is a q x q grid of m x m blocks,
// row (s, a) -> s m + a.  They turn the paper's index reorderings (P-Index,
// P-Index2, Sec. 3, Algorithms 1-2) into address arithmetic of the tile loads
// and epilogue stores.
#pragma once

#include "gemm.h"

namespace ctm {

// W-mix operand: B(k = (s,sg), n = (a,b)) = X[(s m + a) N + sg m + b]
template <class T>
struct B_Mix_ {
    using value_type = T;
    const T *X; int q, m; long Nc;
    static constexpr bool kContigK = false;
    __device__ T operator()(int k, int n) const
    {
        const int s = k / q, sg = k - s * q;
        const int a = n / m, b = n - a * m;
        return X[(long)(s * m + a) * Nc + sg * m + b];
    }
};
using B_Mix = B_Mix_<double>;
using B_Mixf = B_Mix_<float>;
// W-mix store: out(i = (s',sg'), n = (a,b)) -> C[(s' m + a) N + sg' m + b] = acc (times alpha if SCALED;
// the factor is a template switch because a multiply in this epilogue costs the FP64 kernel occupancy)
template <class TO, bool SCALED>
struct EpiMix_ {
    TO *C; int q, m; long Nc; double alpha;
    __device__ void operator()(int i, int n, double v, int) const
    {
        const int sp = i / q, sgp = i - sp * q;
        const int a = n / m, b = n - a * m;
        if constexpr (SCALED) C[(long)(sp * m + a) * Nc + sgp * m + b] = (TO)(alpha * v);
        else C[(long)(sp * m + a) * Nc + sgp * m + b] = (TO)v;
    }
};
// Half-row operand: B(k = gamma, n = (sg, j)) = U[(sg m + gamma) m + j]  (U is N x m)
template <class T>
struct B_Ublk_ {
    using value_type = T;
    const T *U; int m;
    static constexpr bool kContigK = false;
    __device__ T operator()(int k, int n) const
    {
        const int sg = n / m, j = n - sg * m;
        return U[(long)(sg * m + k) * m + j];
    }
};
using B_Ublk = B_Ublk_<double>;
using B_Ublkf = B_Ublk_<float>;

}  // namespace ctm
