// Contractions and fused elementwise kernels of one CTMRG step (Sec. III,
// Algorithm 3 and its Sub-CTMRG), for the state layout described in ctmrg.h.
#pragma once

#include <hip/hip_runtime.h>

namespace ctm {

// Normalization history kept on the device (the log accumulation stays FP64).
struct Book {
    double ln_a, ln_b;     // P_true = a P, C_true = b Omega
    double nC_prev, nC;    // n_C of the previous and the last step
    double nP_prev, nP;    // n_P of the previous and the last step
    double S_prev, S;      // entanglement entropy of the previous and the last step
    double nP_part_max;    // scratch
    int k;                 // steps taken
    int pad;
};

hipError_t build_weight(const double *V, int q, int dim, double K, double *W, double *WH, hipStream_t s);
hipError_t init_state(double *A, double *omega, int q, int m, int bc, int s0, Book *book, hipStream_t s);

// X = A^T diag(omega) A  (N x N), using OA as scratch (m x N)
hipError_t extension_products(const double *A, const double *omega, double *OA, double *X, int q, int m,
                              hipStream_t s);
// Cout_{s' sg'} = sum_{s,sg} W[(s,sg),(s',sg')] Xin_{s sg}   (both N x N, block layout)
hipError_t weight_mix(const double *W, const double *Xin, double *Cout, int q, int m, hipStream_t s);
// Y = A^T [U_1 ... U_q]   (Y[(s,a),(sg,j)] = (P_s U_sg)[a,j])
hipError_t halfrow_products(const double *A, const double *U, double *Y, int q, int m, hipStream_t s);
// Pt = U^T Z  (m x N, the new P in A layout)
// P~ = U^T Z; work (nullable, work_elems doubles) holds split-K partials.
hipError_t projection(const double *U, const double *Z, double *Pt, int q, int m, double *work, size_t work_elems,
                      hipStream_t s);
// Mixed precision (FP32 operands and accumulation on the FP32 matrix cores; with x3, the same
// FP32 operands as three split-bf16 products on the bf16 matrix cores, FP32 accumulation).
// W32 = W / wscale; C' and P~ are produced in FP64 with the factor wscale restored.
hipError_t weight_to_f32(const double *W, float *W32, int q, double wscale, hipStream_t s);
hipError_t state_to_f32(const double *A, const double *omega, float *A32, float *OA32, int q, int m, hipStream_t s);
hipError_t vectors_to_f32(const double *U, float *U32, int q, int m, hipStream_t s);
hipError_t extension_products_f32(const float *A32, const float *OA32, float *X32, int q, int m, bool x3,
                                  hipStream_t s);
hipError_t weight_mix_f32_to_f64(const float *W32, const float *X32, double *Cout, int q, int m, double wscale,
                                 bool x3, hipStream_t s);
hipError_t halfrow_products_f32(const float *A32, const float *U32, float *Y32, int q, int m, bool x3, hipStream_t s);
hipError_t weight_mix_f32(const float *W32, const float *Y32, float *Z32, int q, int m, bool x3, hipStream_t s);
hipError_t projection_f32(const float *U32, const float *Z32, double *Pt, int q, int m, double wscale, double *work,
                          size_t work_elems, bool x3, hipStream_t s);

// n_P = max|Pt|; A = Pt / n_P; book update with n_C (from post), n_P, S_E
hipError_t normalize_and_book(const double *Pt, double *A, int q, int m, double *partials, Book *book,
                              const double *nC_dev, const double *S_dev, hipStream_t s);

// Observables on the current state.  out[0..7]:
//   Z_b, Z_h, Z_d, Z_d[W h4], sum_j w_j^4 (kept), M numerator (fixed: sum_s prob_s v0.v_s),
//   and for free BC the norm of sum_s prob_s v_s in out[5].
hipError_t observables(const double *A, const double *omega, const double *U, const double *W, const double *WH,
                       const double *V, double *OA, double *X, double *H, double *work, size_t work_elems,
                       int q, int dim, int m, int bc, int s0, double *out, hipStream_t s);

}  // namespace ctm
