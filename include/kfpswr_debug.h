/*
 * kfpswr_debug.h -- host-only introspection of libkfpswr's elimination
 * tables, for CPU tests of the planner.  Makes no device call.
 *
 * kfp_debug_tables fills, for a solve of grid g with J subdomains:
 *   sub_info [J][8] ([host]): n, row_off, g_lo, P, lo_kind, hi_kind, tab, seg
 *              (kinds: 0 physical end, 1 Dirichlet interface, 2 Robin row)
 *   rows     [rows][6] ([host]): nu, fa, fb, bc, sl, sr per unknown row
 *   segs     [sum_j (P_j+1)] ([host]): segment starts per subdomain
 *   reds     [sum_j (P_j-1)][5] ([host]): ra, rc, g1, g2, h per separator
 *   mat      [rows][3] ([host]): sub-, main-, super-diagonal per row
 * Capacities: rows from kfp_subdomain_rows, segs J*(waves+1), reds
 * J*waves.  The tables are those a solve with `waves` wavefronts per
 * workgroup uploads.  Returns KFP_EINVAL for invalid arguments.
 */
#ifndef KFPSWR_DEBUG_H
#define KFPSWR_DEBUG_H
#include "kfpswr.h"
#ifdef __cplusplus
extern "C" {
#endif
kfp_status kfp_debug_tables(const kfp_grid *g, int32_t J, int32_t overlap, int32_t tr, double p,
                            int32_t waves, int32_t *sub_info, double *rows, int32_t *segs,
                            double *reds, double *mat);
#ifdef __cplusplus
}
#endif
#endif
