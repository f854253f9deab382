"""Oracle runs for GPU parity tests, in worker processes (test
infrastructure: imports only the oracle and the input generator; no GPU).

Solving several independent problems with the FP64 oracle takes minutes one
after the other; each worker solves one problem on one host thread, so a
pool of the host's cores runs them side by side."""
from __future__ import annotations

import os


def _greedy_job(job):
    from threadpoolctl import threadpool_limits

    from oracle import greedy as ogreedy
    from oracle import operator as oop
    from paper_1808_05510_amd import synth
    kind, gen_kw, opt_kw = job
    with threadpool_limits(limits=1):
        d = synth.box_problem(**gen_kw) if kind == "box" else getattr(synth, kind)(**gen_kw)
        P = oop.problem_from_arrays(d)
        res = ogreedy.greedy_solve(P, ogreedy.GreedyOptions(**opt_kw))
    return res.U, res.Z, res.V, res.history


def greedy_many(jobs, workers=None):
    """Run ogreedy.greedy_solve for every (generator kind, generator kwargs,
    GreedyOptions kwargs) in jobs; returns [(U, Z, V, history)] in order."""
    import concurrent.futures as cf
    import multiprocessing as mp
    workers = workers or max(1, min(16, len(jobs), os.cpu_count() or 1))
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_greedy_job, jobs))
