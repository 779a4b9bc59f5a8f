/*
 * CPU oracle of the learned coarse-grid closure -- TEST INFRASTRUCTURE ONLY.
 * Only tests/, the package's smoke check and the benchmark's CPU baseline may
 * call it; the product path never does.  Plain FP64 definitions.
 */
#ifndef CNN_ORACLE_H
#define CNN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int32_t cnn_param_count(void);
double cnn_bf16(double v);
void cnn_conv3x3(int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout, const double* a, const double* w,
                 const double* bias, double* z);
void cnn_forward(const double* params, int32_t B, int32_t H, int32_t W, const double* x, double* y);
double cnn_loss_grad(const double* params, int32_t B, int32_t H, int32_t W, const double* x, const double* target,
                     double* grad);
void cnn_apply_correction(int32_t nx, int32_t ny, double c, const double* du, const double* dv, double* f);

#ifdef __cplusplus
}
#endif
#endif
