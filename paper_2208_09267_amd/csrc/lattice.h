// lattice.h -- compile-time velocity sets of the GPU library.
//
// D2Q9 follows Table 1 of arXiv:2208.09267 and D3Q27 its Table 2; D3Q19 is
// the rest, face and edge groups of Table 2 with the standard D3Q19 weights
// 1/3, 1/18, 1/36.  The direction order here is this library's own: direction 0 is the
// rest velocity, directions 1..H are a "positive" half and H+1..2H their
// opposites (opp(i) = i +- H), which is what the in-place AA streaming
// pattern swaps between.
#pragma once

namespace vanse {

struct D2Q9 {
    static constexpr int D = 2;
    static constexpr int Q = 9;
    static constexpr int H = 4;
    static constexpr int cx[Q] = {0, 1, 0, 1, -1, -1, 0, -1, 1};
    static constexpr int cy[Q] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
    static constexpr int cz[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                                    1.0 / 36.0, 1.0 / 36.0, 1.0 / 9.0,
                                    1.0 / 9.0,  1.0 / 36.0, 1.0 / 36.0};
};

struct D3Q19 {
    static constexpr int D = 3;
    static constexpr int Q = 19;
    static constexpr int H = 9;
    static constexpr int cx[Q] = {0, 1, 0, 0, 1, 1,  1, 1,  0, 0,
                                  -1, 0, 0, -1, -1, -1, -1, 0, 0};
    static constexpr int cy[Q] = {0, 0, 1, 0, 1, -1, 0, 0,  1, 1,
                                  0, -1, 0, -1, 1,  0, 0,  -1, -1};
    static constexpr int cz[Q] = {0, 0, 0, 1, 0, 0,  1, -1, 1, -1,
                                  0, 0, -1, 0, 0,  -1, 1,  -1, 1};
    static constexpr double w[Q] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                                    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                    1.0 / 36.0, 1.0 / 36.0, 1.0 / 18.0, 1.0 / 18.0,
                                    1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

// D3Q27: Table 2 of the paper (rest 8/27, faces 2/27, edges 1/54, corners
// 1/216); positive half 1..13, opposites 14..26.
struct D3Q27 {
    static constexpr int D = 3;
    static constexpr int Q = 27;
    static constexpr int H = 13;
    static constexpr int cx[Q] = {0, 1, 0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1,
                                  -1, 0, 0, -1, -1, -1, -1, 0, 0, -1, -1, -1, -1};
    static constexpr int cy[Q] = {0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 1, 1, -1, -1,
                                  0, -1, 0, -1, 1, 0, 0, -1, -1, -1, -1, 1, 1};
    static constexpr int cz[Q] = {0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1,
                                  0, 0, -1, 0, 0, -1, 1, -1, 1, -1, 1, -1, 1};
    static constexpr double w[Q] = {
        8.0 / 27.0,  2.0 / 27.0,  2.0 / 27.0,  2.0 / 27.0,  1.0 / 54.0,  1.0 / 54.0,
        1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 216.0, 1.0 / 216.0,
        1.0 / 216.0, 1.0 / 216.0, 2.0 / 27.0,  2.0 / 27.0,  2.0 / 27.0,  1.0 / 54.0,
        1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 54.0,  1.0 / 216.0,
        1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0};
};

template <class L>
__host__ __device__ constexpr int opp(int i)
{
    return i == 0 ? 0 : (i <= L::H ? i + L::H : i - L::H);
}

// Quadrature weight varpi_{i != 0} of the cell integral of phi (Table 3),
// by the number of axes the quadrature runs over (D1Q3, D2Q5, D3Q7).
inline double quad_weight(int n_axes)
{
    return n_axes == 1 ? 1.0 / 4.0 : (n_axes == 2 ? 1.0 / 6.0 : 5.0 / 36.0);
}

}  // namespace vanse
