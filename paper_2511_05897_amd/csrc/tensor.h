// Two-operand contraction through one GEMM (see tensor.hip).
#pragma once
#include "internal.h"
#include <initializer_list>

namespace adc3 {

void ein2(Arena& ws, const char* spec, double alpha, const double* A, const int* adims, const double* B,
          const int* bdims, double beta, double* C, hipStream_t s);

struct TV {  // tensor view: device pointer + dims
    const double* p;
    int d[4];
    TV(const double* ptr, std::initializer_list<int> dims) : p(ptr) {
        int k = 0;
        for (int x : dims) d[k++] = x;
        for (; k < 4; ++k) d[k] = 1;
    }
};
inline void ein(Arena& ws, const char* spec, double alpha, TV A, TV B, double beta, double* C, hipStream_t s) {
    ein2(ws, spec, alpha, A.p, A.d, B.p, B.d, beta, C, s);
}

}  // namespace adc3
