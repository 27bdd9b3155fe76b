// lattice.hpp -- compile-time D3Q7 / D3Q15 / D3Q19 descriptions for the gfx950
// kernels.
//
// Direction vectors and weights of Sec. 3.4, Tables 1 and 2 (same index order
// as the paper).  e^2 = 1/4 for D3Q7 and 1/3 for D3Q15 and D3Q19; for all
// three A_i = delta_{i0} and B_i = w_i - delta_{i0} (Table 2), so the
// supersaturation equilibrium only needs w_i and a rest-population correction.
#pragma once

#include <hip/hip_runtime.h>

namespace lbpf {

struct D3Q7 {
    static constexpr int Q = 7;
    static constexpr double e2 = 1.0 / 4.0;
    __host__ __device__ static constexpr int ex(int i) {
        constexpr int t[7] = {0, 1, 0, -1, 0, 0, 0};
        return t[i];
    }
    __host__ __device__ static constexpr int ey(int i) {
        constexpr int t[7] = {0, 0, 1, 0, -1, 0, 0};
        return t[i];
    }
    __host__ __device__ static constexpr int ez(int i) {
        constexpr int t[7] = {0, 0, 0, 0, 0, 1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr double w(int i) { return i == 0 ? 1.0 / 4.0 : 1.0 / 8.0; }
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr double e2 = 1.0 / 3.0;
    __host__ __device__ static constexpr int ex(int i) {
        constexpr int t[19] = {0, 1, 0, -1, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
        return t[i];
    }
    __host__ __device__ static constexpr int ey(int i) {
        constexpr int t[19] = {0, 0, 1, 0, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr int ez(int i) {
        constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
};

struct D3Q15 {
    static constexpr int Q = 15;
    static constexpr double e2 = 1.0 / 3.0;
    __host__ __device__ static constexpr int ex(int i) {
        constexpr int t[15] = {0, 1, 0, -1, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
        return t[i];
    }
    __host__ __device__ static constexpr int ey(int i) {
        constexpr int t[15] = {0, 0, 1, 0, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr int ez(int i) {
        constexpr int t[15] = {0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
        return t[i];
    }
    __host__ __device__ static constexpr double w(int i) {
        return i == 0 ? 2.0 / 9.0 : (i < 7 ? 1.0 / 9.0 : 1.0 / 72.0);
    }
};

// e^2 of the lattice with q populations (Table 2).
inline double lattice_e2(int q) { return q == 7 ? D3Q7::e2 : D3Q19::e2; }

// Index of the direction (x,y,z) in lattice L, -1 if none.  Evaluated on the
// device only for links that cross a wall.
template <class L>
__host__ __device__ inline int find_dir(int x, int y, int z) {
    int r = -1;
#pragma unroll
    for (int i = 0; i < L::Q; ++i)
        if (L::ex(i) == x && L::ey(i) == y && L::ez(i) == z) r = i;
    return r;
}

}  // namespace lbpf
