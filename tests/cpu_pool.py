"""CPU work of the GPU tests in fresh worker processes (test helper): the FP64
oracle's ADMM for several slices in parallel, and the synthesis of whole workloads
(which forks its own workers).  The workers are started with the spawn method, so
no process that has initialised the GPU is ever forked; oracle workers use one
BLAS thread each."""

import contextlib
import os

_THREAD_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")


def _admm_job(job):
    from oracle import t2s as O
    ksp, sens, phi, masks, kw = job
    return O.admm(ksp, sens, phi, masks, **kw).alpha


def _config_job(conn, name, kw):
    from synth import make_config
    conn.send(make_config(name, **kw))
    conn.close()


@contextlib.contextmanager
def _env(**kv):
    old = {v: os.environ.get(v) for v in kv}
    os.environ.update(kv)
    try:
        yield
    finally:
        for v, x in old.items():
            if x is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = x


def admm_many(jobs, procs=16):
    """jobs: list of (samples, sens, phi, masks, admm keyword arguments); returns the
    list of FP64 alpha arrays in job order."""
    import multiprocessing as mp
    with _env(**{v: "1" for v in _THREAD_VARS}):
        ctx = mp.get_context("spawn")
        with ctx.Pool(max(1, min(len(jobs), procs, os.cpu_count() or 1))) as pool:
            return pool.map(_admm_job, jobs)


def make_config_spawned(name, **kw):
    """synth.make_config(name, **kw), run in a fresh (non-daemonic) process, which
    may fork its own synthesis workers."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    recv, send = ctx.Pipe(duplex=False)
    proc = ctx.Process(target=_config_job, args=(send, name, kw))
    proc.start()
    send.close()
    try:
        out = recv.recv()
    finally:
        proc.join()
    if proc.exitcode != 0:
        raise RuntimeError(f"workload synthesis failed (exit code {proc.exitcode})")
    return out
