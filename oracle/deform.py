"""Deformation update of the reduced system (eq. problem:2, Sec. 4.2): the
deformation equation only involves the mass matrix on both sides, so the
update is one vector addition of the condensation relation (Sec. 3.1)

    u_n = u_{n-1} + k theta v_n + k (1 - theta) v_{n-1}

at interface and solid nodes.  For a Newton increment (u_{n-1}, v_{n-1}
fixed) this is du = k theta dv.  Entries at nodes outside the mask are set to
zero: there the deformation is the ALE extension (eq. problem:3)."""
import numpy as np


def deform_update(mask_nodes, k, theta, v_new, u_old=None, v_old=None):
    """mask_nodes: bool [nnodes]; v_new, u_old, v_old: [nnodes, d] (None = 0)."""
    v_new = np.asarray(v_new, dtype=np.float64)
    u = k * theta * v_new
    if u_old is not None:
        u = u + u_old
    if v_old is not None:
        u = u + k * (1.0 - theta) * v_old
    out = np.zeros_like(v_new)
    out[mask_nodes] = u[mask_nodes]
    return out
