/*
 * emu_host.h -- host-only view of the EMU mesh setup (no GPU needed).
 *
 * Runs the same setup as emu_create_mesh (validation, orientation, ACAP weights,
 * weighted Laplacian L_w of eq. ACAPEnergy, nested-dissection ordering,
 * supernodal factorization of L_ff, lowest eigenpairs of eq. low-rank) entirely
 * on the host, and exposes the factor and modes so they can be checked against
 * independent sparse solvers.  Same conventions as emu.h: host pointers only,
 * user vertex numbering, EMU_OK or an error code, message in emu_last_error().
 */
#ifndef EMU_HOST_H
#define EMU_HOST_H

#include "emu.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct emu_host_setup emu_host_setup;

emu_status emu_host_setup_create(const emu_mesh_desc* desc, emu_host_setup** out);
emu_status emu_host_setup_destroy(emu_host_setup* s);
emu_status emu_host_setup_info(const emu_host_setup* s, emu_mesh_info* info);

/* x = L_ff^{-1} b per coordinate.  b, x: host [n][3]; rows of pinned vertices
   are ignored in b and set to 0 in x. */
emu_status emu_host_setup_solve(const emu_host_setup* s, const double* b, double* x);

/* y = L_w x over all vertices (host [n][3] each): the assembled operator. */
emu_status emu_host_setup_apply(const emu_host_setup* s, const double* x, double* y);

/* Lowest k/3 eigenpairs of L_ff: nu host [k1], phi host [k1][n] (zero at pins). */
emu_status emu_host_setup_modes(const emu_host_setup* s, double* nu, double* phi);

/* Oriented tets (host [m][4]), volumes [m] and ACAP weights [m]; any may be NULL. */
emu_status emu_host_setup_geometry(const emu_host_setup* s, int32_t* tets, double* vol, double* w);

#ifdef __cplusplus
}
#endif
#endif /* EMU_HOST_H */
