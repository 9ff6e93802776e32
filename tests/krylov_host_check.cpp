// C entry points over the host-side s-step GMRES helper, built with g++ by
// tests/test_krylov_host.py (the header has no HIP dependency).
#include "../paper_2112_05051_amd/csrc/krylov_host.hpp"

extern "C" {
int kh_leja_order(const double *pts, int n, int k, double *out) { return rich::leja_order(pts, n, k, out); }
void kh_leja_points(double a, double b, int k, double *out) { rich::leja_points(a, b, k, out); }
}
