"""Adapters from the input generator's level data to fsimg level descriptors
(argument marshalling: arrays are passed as they are)."""


def level_dicts(problem, system: str, with_class: bool = True):
    """Per-level descriptor dicts (finest first) of one system ("mom", "ale"
    or "mass") of an fsigen.Problem."""
    out = []
    for lev in problem.levels:
        m = lev.systems[system]
        out.append(dict(dim=lev.dim, block=m.b, cells=list(lev.cells), rowptr=m.rowptr,
                        colind=m.colind, vals=m.vals, dirichlet=m.dirichlet,
                        cell_class=lev.cell_solid if with_class else None))
    return out


def request_data(problem, states=(), rhs=()):
    """fsimg.RequestData (momentum + ALE) of an fsigen.Problem; `states` are
    further problems on the same mesh whose momentum values are cycled over
    the time steps, `rhs` further momentum right-hand sides cycled over the
    Newton steps."""
    from .fsimg import RequestData
    fine = problem.levels[0]
    vals = [[lv.systems["mom"].vals for lv in st.levels] for st in states]
    return RequestData(level_dicts(problem, "mom"), level_dicts(problem, "ale"), problem.rhs["mom"],
                       problem.rhs["ale"], fine.node_solid, problem.params["k"],
                       problem.params["theta"], states=vals, rhs=list(rhs))


def fsi_levels(problem):
    """Per-level geometry (coordinates per axis, cell_solid, node positions
    or None) for fsimg.fsimg_fsi_create."""
    return [(list(lev.coords), lev.cell_solid, lev.node_coords) for lev in problem.levels]


def fsi_state(problem):
    """The generator's state as Newton-loop vectors (node-major FP64 numpy):
    x = (p = 0, v_cur), u_cur, x_old = (0, v_old), u_old."""
    import numpy as np
    n, d = problem.levels[0].nnodes, problem.dim
    x = np.zeros((n, d + 1))
    x[:, 1:] = problem.v_cur
    xo = np.zeros((n, d + 1))
    xo[:, 1:] = problem.v_old
    return (x.ravel(), np.ascontiguousarray(problem.u_cur).ravel(), xo.ravel(),
            np.ascontiguousarray(problem.u_old).ravel())
