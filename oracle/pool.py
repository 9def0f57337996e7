"""Several independent oracle propagator solves at once, one per worker process.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The solves of different
sources share nothing, so they run in separate processes; each worker calls
``redblack.propagator`` unchanged.  Workers are started with the "spawn" method, so
they never inherit a GPU context of the calling process.
"""

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

from . import redblack


def _solve(U, eta, p, tol, form):
    if form is None:
        return redblack.propagator(U, eta, p, tol=tol)
    return redblack.propagator_form(U, eta, p, form, tol=tol)


def _one(args):
    U, eta, p, tol, form = args
    try:  # one BLAS thread per worker: the workers already fill the cores
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            y, info = _solve(U, eta, p, tol, form)
    except ImportError:
        y, info = _solve(U, eta, p, tol, form)
    return y, info.iters


def propagators(U, etas, p, tol=1e-10, workers=None, forms=None):
    """[(y_1, CGLS iterations)] of redblack.propagator for each source in etas, or of
    redblack.propagator_form with forms[i] for source i."""
    forms = [None] * len(etas) if forms is None else list(forms)
    jobs = [(U, e, p, tol, f) for e, f in zip(etas, forms)]
    if workers is None:
        workers = min(len(jobs), len(os.sched_getaffinity(0)), 16)
    if workers <= 1:
        return [_one(j) for j in jobs]
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_one, jobs))
