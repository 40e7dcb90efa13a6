// Per-right-hand-side Krylov scalars kept on the device (solver.hip; read by the fused
// hopping epilogue of the multi-RHS kernel).
#pragma once

#include <hip/hip_runtime.h>

// most directions whose steps the CG or BiCGStab solution increment may still owe (the
// current one included)
constexpr int kMaxDirs = 8;

struct Scal {
    double2 rho, alpha, omega, beta;
    double2 aux;      // <r, p> / |r|^2 after a reliable update (CG)
    double rho_prev;  // |r|^2 of the previous CG iteration
    double r2;        // |r|^2 of the iterated residual
    double r2hi;      // |r|^2 of the last FP64 residual
    double tol2;      // target |r|^2 of the even-odd system
    double b2;        // |bhat|^2
    double alpha_prev[kMaxDirs - 1];  // alpha of the previous CG iterations, latest first (steps
                                      // the direction update still owes x)
    double2 bs_alpha_prev[kMaxDirs - 1];  // the same for BiCGStab: alpha and omega of the
    double2 bs_omega_prev[kMaxDirs - 1];  // previous iterations, latest first
    int active;
    int iters;
    int breakdown;
    int pad;
};
