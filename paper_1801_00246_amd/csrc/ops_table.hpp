// Reference operators of one degree packed in the order of OpsLayout<N>:
// D_r, D_s, M D_r, M D_s, M, M^{-1}, LIFT, face mass.
#pragma once
#include <vector>

namespace ipdg {
std::vector<double> build_ops_table(int N);
}
