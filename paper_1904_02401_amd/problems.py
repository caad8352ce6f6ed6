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


def request_data(problem):
    """fsimg.RequestData (momentum + ALE) of an fsigen.Problem."""
    from .fsimg import RequestData
    fine = problem.levels[0]
    return RequestData(level_dicts(problem, "mom"), level_dicts(problem, "ale"), problem.rhs["mom"],
                       problem.rhs["ale"], fine.node_solid, problem.params["k"],
                       problem.params["theta"])
