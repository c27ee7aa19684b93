// Internal layout of a PDF grid on the device (shared by pdf.hip and the
// fused t tbar integrand).
#pragma once

#include "common.h"

#define VGX_MAX_SUB 8
#define VGX_MAX_FLAV 16

struct vgx_pdf {
  int device = 0;
  int n_x = 0, n_sub = 0, n_flav = 0;
  int n_members = 1;                  // members of a PDF set (shared knots), member-major values
  int fstride = 0;                    // node stride (= n_flav)
  int extrap = VGX_EXTRAP_ERROR;      // behaviour outside the grid (pdf_interp, pdf_alphas)
  int nq[VGX_MAX_SUB] = {0};
  int q_off[VGX_MAX_SUB + 1] = {0};   // knot offset of each subgrid
  // host copies (knots only; values stay on the device)
  double* h_x = nullptr;              // [n_x]
  double* h_q2 = nullptr;             // [q_off[n_sub]]
  // device arrays
  double* x = nullptr;                // [n_x]            x knots
  double* lx = nullptr;               // [n_x]            ln x knots
  double* q2 = nullptr;               // [total q]        Q^2 knots
  double* lq2 = nullptr;              // [total q]        ln Q^2 knots
  double* v64 = nullptr;              // [member][total q][n_x][fstride]  node values (FP64); member 0
                                      // is what pdf_interp and the fused integrands read
  float* v32 = nullptr;               // same, FP32 copy
  unsigned long long* oor = nullptr;  // out-of-range counter
  // alpha_s(Q) table (optional; pdf_set_alphas): knots on the Q^2 line split
  // into subgrids at duplicated knots
  int a_nsub = 0;
  int a_nq[VGX_MAX_SUB] = {0};
  int a_off[VGX_MAX_SUB + 1] = {0};
  double* h_aq2 = nullptr;            // host [total] knots
  double* h_aval = nullptr;           // host [total] values
  double* a_lq2 = nullptr;            // device [total] ln Q^2 knots
  double* a_val = nullptr;            // device [total] values
};
