"""Shared helpers of the GPU parity tests: run the same seeded case through
the HIP library and through the CPU oracle."""
import sys

import numpy as np

import oracle
import workloads

_OKIND = {1: oracle.D1Q7, 2: oracle.D2Q49, 3: oracle.D3Q343}
_ONAMED = {"D2Q37": oracle.D2Q37}


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_run(shape, bc, n_rot, tau, dtype, fields, steps, perturb_seed=None, tile=None,
            graphs=True, chunks=None, inplace=None, blocked=None, lattice=None, fd=None, g_substeps=1):
    """Populations come back in the library's slot order (lattice_info)."""
    import torch
    from paper_1606_06107_amd import Sim
    sim = Sim(shape, bc=bc, n_rot=n_rot, tau=tau, dtype=dtype, lattice=lattice,
              g_substeps=g_substeps).init(*fields)
    if fd is not None:
        sim.set_fd(fd)
    if perturb_seed is not None:
        f, g = sim.populations()
        pf = torch.as_tensor(workloads.nonequilibrium_perturbation(f.shape, perturb_seed)).to(f)
        pg = torch.as_tensor(workloads.nonequilibrium_perturbation(g.shape, perturb_seed + 1)).to(g)
        sim.init_populations(f * pf, g * pg)
    if blocked is not None:
        sim.set_blocked(blocked)
    if tile is not None:
        sim.set_tile(*tile)
    if inplace is not None:
        sim.set_inplace(inplace)
    sim.set_graphs(graphs)
    for k in (chunks or [steps]):
        sim.step(k)
    rho, u, T, tot = sim.moments()
    f, g = sim.populations()
    torch.cuda.synchronize()
    return {"rho": rho.cpu().numpy(), "u": u.cpu().numpy(), "T": T.cpu().numpy(),
            "tot": tot.cpu().numpy(), "f": f.double().cpu().numpy(), "g": g.double().cpu().numpy()}


def oracle_run(shape, bc, n_rot, tau, fields, steps, perturb_seed=None, lattice=None, fd=0.0, g_substeps=1):
    """Populations come back in the oracle's order (oracle.lattice)."""
    D = len(shape)
    obc = [oracle.OPEN if b == "open" else oracle.PERIODIC for b in bc]
    G = oracle.Grid(_ONAMED[lattice] if lattice else _OKIND[D], shape, bc=obc, n_rot=n_rot, tau=tau,
                    fd_courant=fd, g_substeps=g_substeps)
    f, g = G.init_eq(*fields)
    if perturb_seed is not None:
        f *= workloads.nonequilibrium_perturbation(f.shape, perturb_seed)
        g *= workloads.nonequilibrium_perturbation(g.shape, perturb_seed + 1)
    G.step(f, g, steps)
    rho, u, T, tot = G.moments(f, g)
    return {"rho": rho, "u": u, "T": T, "tot": tot, "f": f, "g": g}


def rel_err(a, b):
    """max |a - b| / max |b| (normwise relative, FP64 parity measure)."""
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def field_err(key, a, b, T_ref):
    """Normwise relative error of one field.  u is a difference quantity
    (sum c f) whose rounding scales with the sound speed, so it is measured
    against max(max|u|, sqrt(max T))."""
    a, b = np.asarray(a), np.asarray(b)
    scale = np.abs(b).max()
    if key == "u":
        scale = max(scale, float(np.sqrt(np.abs(T_ref).max())))
    return float(np.abs(a - b).max() / max(scale, 1e-300))


def abs_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())


def smooth_fields(shape, seed, mach=0.3, gamma=1.4):
    """The 2-D periodic workload's recipe at another size (1-D and 3-D use
    the same mode sums)."""
    if len(shape) == 2:
        w = workloads.Periodic2D(nx=shape[0], ny=shape[1], gamma=gamma, mach=mach, seed=seed)
        return w.fields()
    rng = np.random.default_rng(seed)
    N = int(np.prod(shape))
    D = len(shape)
    grids = np.meshgrid(*[np.arange(n) / n for n in shape[::-1]], indexing="ij")
    def modes(r):
        out = np.zeros(grids[0].shape)
        for _ in range(4):
            k = r.integers(-2, 3, D)
            out += r.uniform(0.1, 0.3) * np.cos(2 * np.pi * sum(k[d] * grids[d] for d in range(D)) + r.uniform(0, 6.3))
        return out.reshape(-1)
    rho = 1 + 0.05 * modes(rng)
    u = np.stack([0.15 * modes(rng) for _ in range(D)])
    T = 1 + 0.05 * modes(rng)
    return rho, u, T


def slot_permutation(c_lib, c_orc):
    """perm with c_orc[perm[s]] == c_lib[s]: oracle rows in library slot order."""
    index = {tuple(int(v) for v in row[:2]): k for k, row in enumerate(np.asarray(c_orc))}
    return np.array([index[tuple(int(v) for v in row[:2])] for row in np.asarray(c_lib)])
