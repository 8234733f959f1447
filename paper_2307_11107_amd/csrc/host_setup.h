// Host-side FP64 set-up of a grain (geometry tables and multigrid operators).
#pragma once
#include <array>
#include <vector>

namespace apic {

enum { ST_C = 0, ST_W, ST_E, ST_S, ST_N, ST_SW, ST_SE, ST_NW, ST_NE, ST_COUNT };

// 9-point stencil over all nodes of an n1 x n2 grid (rows on the Dirichlet
// columns are zero); nn / ss hold the second-neighbour coefficient of the axis
// rows on the finest level (empty on coarse levels).
struct Stencil {
    int n1 = 0, n2 = 0;
    std::array<std::vector<double>, ST_COUNT> c;
    std::vector<double> nn, ss;
};

void node_volumes(int n1, int n2, double x1_out, double alpha, std::vector<double>& vol);
double outer_area(double x1_out, double alpha);
double bound_volume_marginal(double x1_out, double alpha);
double bound_outer_area_density(double x1_out, double alpha);
double grain_max_radius(double alpha);
void fine_stencil(int n1, int n2, double x1_out, double alpha, Stencil& s);
void fine_stencil_fe(int n1, int n2, double x1_out, double alpha, Stencil& s);
void galerkin_coarse(const Stencil& fine, Stencil& coarse);
void dense_matrix(const Stencil& s, std::vector<double>& A);
bool invert(std::vector<double> A, int m, std::vector<double>& inv, int threads);
double boundary_coupling_norm2(const Stencil& s, double phi_grain, double phi_out);

}  // namespace apic
