// Host build of the library's FP64 exp/log for the accuracy test.
#include "rt_math.hpp"

extern "C" void rt_exp_many(const double* x, double* y, long n) {
    for (long i = 0; i < n; ++i) y[i] = rtk::rt_exp(x[i]);
}
extern "C" void rt_log_many(const double* x, double* y, long n) {
    for (long i = 0; i < n; ++i) y[i] = rtk::rt_log(x[i]);
}
