"""Helpers shared by the GPU parity tests: same seeded inputs to both sides."""
import numpy as np

import workloads as wl


def random_env(Lx, Ly, chi, Db, seed):
    """Random corners / edges (all legs chi) for every site: list of (C[4], T[4])."""
    return wl.random_environment(Lx, Ly, chi, Db, seed)


def inject(oracle_env, gpu_ctx, env):
    for i, (C, T) in enumerate(env):
        oracle_env.C[i] = [c.copy() for c in C]
        oracle_env.T[i] = [t.copy() for t in T]
        if gpu_ctx is not None:
            gpu_ctx.ctm_set_env(i, C, T)


def ulp_perturbed(tensors, seed):
    """Every entry moved one unit in the last place, up or down at random: a
    change of the inputs at the level of unit roundoff, whose effect on a run
    is the run's own sensitivity to rounding."""
    rng = np.random.default_rng(seed)
    out = []
    for a in tensors:
        a = np.asarray(a, dtype=np.float64)
        up = rng.random(a.shape) < 0.5
        out.append(np.where(up, np.nextafter(a, np.inf), np.nextafter(a, -np.inf)))
    return out


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def pad_to(x, shape):
    out = np.zeros(shape)
    out[tuple(slice(0, s) for s in x.shape)] = x
    return out


def load_state(gpu_ctx, oracle_env):
    """Copy the oracle's environment (any bond dimensions up to chi) into the
    GPU context, zero padded, with its dimensions."""
    chi, Db = gpu_ctx.chi, gpu_ctx.Db
    for i in range(len(oracle_env.C)):
        C, T = oracle_env.C[i], oracle_env.T[i]
        dims = [list(C[k].shape) for k in range(4)] + [list(T[k].shape[:2]) for k in range(4)]
        gpu_ctx.ctm_set_env(i, [pad_to(c, (chi, chi)) for c in C], [pad_to(t, (chi, chi, Db)) for t in T],
                            np.array(dims, dtype=np.int32))
