"""Synthetic T2-Shuffling acquisitions (scanner simulation, not reconstruction).

Recipes (all seeded with numpy PCG64):

* Basis: echo times TE_t = (t + 1) * ESP (ESP = 6 ms), 1000 T2 values on a uniform
  grid in [20, 300] ms, signals exp(-TE / T2); Phi = the K leading left singular
  vectors of that T x 1000 matrix, each column signed so its largest-magnitude
  entry is positive.  Returned as float32 [T, K].
* Phantom: 6 ellipses (2D) or ellipsoids (3D, sliced along the readout axis),
  painted in order (later ones overwrite), background 0, real valued.  Centres in
  the central 80 % of the field of view, semi-axes U[0.1, 0.4] * FOV, random
  rotation; proton density U[0.2, 1], T2 U[20, 300] ms.  Echo image
  x_t = PD * exp(-TE_t / T2) inside each region.
* Coils: C Gaussian bumps (sigma = 0.4 FOV) centred on a circle (2D) or on rings
  of a cylinder around the readout axis (3D) of radius 0.6 FOV, constant phase
  2 pi c / C, divided by their root-sum-of-squares so that sum_c |S_c|^2 = 1.
* Masks: per echo an independent variable-density Poisson-disc pattern made by
  greedy dart throwing on the integer grid.  Candidates are visited in a random
  order weighted towards the centre; a candidate is accepted if no accepted point
  lies within d(r) = d0 (1 + 2 r) (r = normalised distance from DC); d0 is set so
  the packing capacity is about 1.3x the target count and the throwing stops at
  the target count.  DC is always sampled by at least one echo; optionally every
  point of a central ellipse of a given area fraction is covered by the union of
  the echoes (missing points go to a random echo).
* Samples: the centred unitary 2D DFT of S_c x_t at the sampled locations, in mask
  order (echo-major, then row-major (y, z) position inside mask_t), plus circular
  complex Gaussian noise at a linear amplitude SNR ||y_clean|| / ||w|| over the
  sampled entries of each slice.

Per-slice data depend only on (config seed, slice index), so any subset of slices
of a volume is generated bit-identically to the same slices of the full volume.
"""

from __future__ import annotations

import dataclasses
import mmap
import multiprocessing as mp
import os

import numpy as np
import scipy.fft as sfft

ESP_MS = 6.0

# ---------------------------------------------------------------------------
# Workload descriptions (shapes and schedules of the five workloads), by name
# ---------------------------------------------------------------------------

CONFIGS = {
    "slice64_c4_t16_k3": dict(name="slice64_c4_t16_k3", classes=[dict(ny=64, nz=64, ncoils=4, nslices=1, nx=1)],
            T=16, K=3, frac=0.04, center_frac=None, snr=30.0, dims=2, lam=0.01, rho=0.1, block=8,
            n_outer=20, n_cg=5, tol=0.0, seed=0),
    "vol320_256x256_c8_t80_k4": dict(name="vol320_256x256_c8_t80_k4", classes=[dict(ny=256, nz=256, ncoils=8, nslices=320, nx=320)],
            T=80, K=4, frac=0.015, center_frac=0.10, snr=30.0, dims=3, lam=0.01, rho=0.1, block=8,
            n_outer=100, n_cg=5, tol=0.0, seed=1),
    "mixed48_192c6_256c8_320x256c12_t80_k4": dict(name="mixed48_192c6_256c8_320x256c12_t80_k4",
            classes=[dict(ny=192, nz=192, ncoils=6, nslices=16, nx=256, seed=2),
                     dict(ny=256, nz=256, ncoils=8, nslices=16, nx=256, seed=3),
                     dict(ny=320, nz=256, ncoils=12, nslices=16, nx=256, seed=4)],
            T=80, K=4, frac=0.015, center_frac=0.10, snr=30.0, dims=3, lam=0.01, rho=0.1, block=8,
            n_outer=100, n_cg=5, tol=0.0, seed=2),
    "warmstart_eval320_256x256_c8_t80_k4": dict(name="warmstart_eval320_256x256_c8_t80_k4", classes=[dict(ny=256, nz=256, ncoils=8, nslices=320, nx=320)],
            T=80, K=4, frac=0.015, center_frac=0.10, snr=30.0, dims=3, lam=0.01, rho=0.1, block=8,
            n_outer=500, n_cg=5, tol=1e-4, seed=11),
    "vol512_384x384_c16_t100_k5": dict(name="vol512_384x384_c16_t100_k5", classes=[dict(ny=384, nz=384, ncoils=16, nslices=512, nx=512)],
            T=100, K=5, frac=0.01, center_frac=0.10, snr=30.0, dims=3, lam=0.01, rho=0.1, block=8,
            n_outer=500, n_cg=5, tol=1e-4, seed=5),
}


# ---------------------------------------------------------------------------
# Basis
# ---------------------------------------------------------------------------


def basis(T: int, K: int, esp_ms: float = ESP_MS, t2_lo: float = 20.0, t2_hi: float = 300.0,
          n_t2: int = 1000) -> np.ndarray:
    te = (np.arange(T) + 1.0) * esp_ms
    t2 = np.linspace(t2_lo, t2_hi, n_t2)
    sig = np.exp(-te[:, None] / t2[None, :])
    U, _, _ = np.linalg.svd(sig, full_matrices=False)
    phi = U[:, :K].copy()
    for k in range(K):
        if phi[np.argmax(np.abs(phi[:, k])), k] < 0:
            phi[:, k] = -phi[:, k]
    return phi.astype(np.float32)


def echo_times(T: int, esp_ms: float = ESP_MS) -> np.ndarray:
    return (np.arange(T) + 1.0) * esp_ms


# ---------------------------------------------------------------------------
# Phantoms
# ---------------------------------------------------------------------------


def _grid(n):
    return (np.arange(n) - n // 2) / n          # normalised coordinate in [-0.5, 0.5)


def draw_ellipses(rng, n=6):
    """2D ellipses: centre, semi-axes, angle, PD, T2."""
    out = []
    for _ in range(n):
        out.append(dict(c=rng.uniform(-0.4, 0.4, 2), ax=rng.uniform(0.1, 0.4, 2),
                        ang=rng.uniform(0.0, np.pi), pd=rng.uniform(0.2, 1.0), t2=rng.uniform(20.0, 300.0)))
    return out


def labels_2d(ells, ny, nz):
    y = _grid(ny)[:, None]
    z = _grid(nz)[None, :]
    lab = np.zeros((ny, nz), dtype=np.int32)
    for i, e in enumerate(ells):
        ca, sa = np.cos(e["ang"]), np.sin(e["ang"])
        dy, dz = y - e["c"][0], z - e["c"][1]
        u = (ca * dy + sa * dz) / e["ax"][0]
        v = (-sa * dy + ca * dz) / e["ax"][1]
        lab[u * u + v * v <= 1.0] = i + 1
    return lab


def _rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def draw_ellipsoids(rng, n=6):
    out = []
    for _ in range(n):
        out.append(dict(c=rng.uniform(-0.4, 0.4, 3), ax=rng.uniform(0.1, 0.4, 3), R=_rotation(rng),
                        pd=rng.uniform(0.2, 1.0), t2=rng.uniform(20.0, 300.0)))
    return out


def labels_3d_slice(ells, nx, ix, ny, nz):
    """Label image of readout slice ix (coordinates x, y, z; slice plane = (y, z))."""
    x = _grid(nx)[ix]
    y = _grid(ny)[:, None]
    z = _grid(nz)[None, :]
    lab = np.zeros((ny, nz), dtype=np.int32)
    for i, e in enumerate(ells):
        d = (x - e["c"][0], y - e["c"][1], z - e["c"][2])
        acc = 0.0
        for a in range(3):
            comp = e["R"][0, a] * d[0] + e["R"][1, a] * d[1] + e["R"][2, a] * d[2]
            acc = acc + (comp / e["ax"][a]) ** 2
        lab[acc <= 1.0] = i + 1
    return lab


# ---------------------------------------------------------------------------
# Coil maps
# ---------------------------------------------------------------------------


def coils_2d(C, ny, nz, rot=0.0):
    y = _grid(ny)[:, None]
    z = _grid(nz)[None, :]
    g = np.empty((C, ny, nz), dtype=np.complex128)
    for c in range(C):
        th = 2 * np.pi * c / C + rot
        cy, cz = 0.6 * np.cos(th), 0.6 * np.sin(th)
        g[c] = np.exp(-((y - cy) ** 2 + (z - cz) ** 2) / (2 * 0.4 ** 2)) * np.exp(1j * 2 * np.pi * c / C)
    g /= np.sqrt(np.sum(np.abs(g) ** 2, axis=0))[None]
    return g.astype(np.complex64)


def coils_3d_slice(C, nx, ix, ny, nz):
    rings = 2 if C >= 8 else 1
    per = C // rings
    x = _grid(nx)[ix]
    y = _grid(ny)[:, None]
    z = _grid(nz)[None, :]
    g = np.empty((C, ny, nz), dtype=np.complex128)
    for c in range(C):
        ring, j = divmod(c, per) if c < rings * per else (rings - 1, c - (rings - 1) * per)
        th = 2 * np.pi * j / per + (np.pi / per) * ring
        cx = 0.0 if rings == 1 else (-0.2 if ring == 0 else 0.2)
        cy, cz = 0.6 * np.cos(th), 0.6 * np.sin(th)
        g[c] = (np.exp(-((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) / (2 * 0.4 ** 2))
                * np.exp(1j * 2 * np.pi * c / C))
    g /= np.sqrt(np.sum(np.abs(g) ** 2, axis=0))[None]
    return g.astype(np.complex64)


# ---------------------------------------------------------------------------
# Variable-density Poisson-disc masks
# ---------------------------------------------------------------------------


def _disk_offsets(rmax):
    r = int(np.ceil(rmax))
    dy, dz = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1), indexing="ij")
    d2 = dy * dy + dz * dz
    keep = d2 > 0
    order = np.argsort(d2[keep], kind="stable")
    return dy[keep][order], dz[keep][order], d2[keep][order]


def _one_mask(rng, ny, nz, target):
    ky = (np.arange(ny) - ny // 2) / (ny / 2)
    kz = (np.arange(nz) - nz // 2) / (nz / 2)
    rr = np.sqrt(ky[:, None] ** 2 + kz[None, :] ** 2) / np.sqrt(2.0)
    shape = (1.0 + 2.0 * rr)
    dens = 1.0 / shape ** 2
    d0 = np.sqrt(0.7 * dens.sum() / (1.3 * target))
    # weighted random visiting order (Efraimidis-Spirakis keys)
    keys = np.log(rng.random(ny * nz)) / dens.reshape(-1)
    order = np.argsort(-keys, kind="stable")
    occ = np.zeros((ny, nz), dtype=bool)
    count = 0
    while count < target:
        dmax = d0 * 3.0
        oy, oz, od2 = _disk_offsets(dmax)
        dlim = (d0 * shape.reshape(-1)) ** 2
        for n in order:
            if count >= target:
                break
            y, z = divmod(int(n), nz)
            if occ[y, z]:
                continue
            lim = dlim[n]
            sel = od2 < lim
            yy = y + oy[sel]
            zz = z + oz[sel]
            ok = (yy >= 0) & (yy < ny) & (zz >= 0) & (zz < nz)
            if occ[yy[ok], zz[ok]].any():
                continue
            occ[y, z] = True
            count += 1
        d0 *= 0.85                               # saturated before the target: tighten and continue
    return occ


def vd_poisson_masks(seed, T, ny, nz, frac, center_frac=None):
    """T independent VD Poisson-disc masks, uint8 [T, ny, nz], centred (DC at (ny/2, nz/2))."""
    rng = np.random.default_rng([seed, 7])
    target = max(1, int(round(frac * ny * nz)))
    masks = np.stack([_one_mask(rng, ny, nz, target) for _ in range(T)])
    if not masks[:, ny // 2, nz // 2].any():
        masks[0, ny // 2, nz // 2] = True
    if center_frac:
        s = np.sqrt(center_frac / np.pi)
        ky = (np.arange(ny) - ny // 2) / (ny * s)
        kz = (np.arange(nz) - nz // 2) / (nz * s)
        inside = ky[:, None] ** 2 + kz[None, :] ** 2 <= 1.0
        missing = np.argwhere(inside & ~masks.any(axis=0))
        if len(missing):
            echo = rng.integers(0, T, len(missing))
            masks[echo, missing[:, 0], missing[:, 1]] = True
    return masks.astype(np.uint8)


# ---------------------------------------------------------------------------
# Acquisition
# ---------------------------------------------------------------------------


def _fft2c(x):
    ax = (-2, -1)
    workers = 1 if mp.current_process().name != "MainProcess" else min(16, os.cpu_count() or 1)
    return sfft.fftshift(sfft.fft2(sfft.ifftshift(x, axes=ax), axes=ax, norm="ortho", workers=workers), axes=ax)


def sample_locations(masks):
    """(echo index, flat location) of every sample, in mask order."""
    t_idx, loc = [], []
    for t in range(masks.shape[0]):
        flat = np.flatnonzero(masks[t].reshape(-1))
        t_idx.append(np.full(flat.size, t, dtype=np.int64))
        loc.append(flat)
    return np.concatenate(t_idx), np.concatenate(loc)


def acquire(labels, pd, t2, sens, masks, snr, rng, esp_ms=ESP_MS, locs=None):
    """Noisy k-space samples [C, P_tot] (complex64) of the echo images of a labelled phantom."""
    T = masks.shape[0]
    C, ny, nz = sens.shape
    t_of, loc = locs if locs is not None else sample_locations(masks)
    te = echo_times(T, esp_ms)
    regions = [r for r in range(1, len(pd) + 1) if np.any(labels == r)]
    out = np.zeros((C, t_of.size), dtype=np.complex128)
    if regions:
        ind = np.stack([(labels == r) for r in regions]).astype(np.complex128)     # [R, ny, nz]
        G = _fft2c(ind[:, None] * sens.astype(np.complex128)[None])                # [R, C, ny, nz]
        G = G.reshape(len(regions), C, ny * nz)[:, :, loc]                           # [R, C, P]
        e = np.stack([pd[r - 1] * np.exp(-te / t2[r - 1]) for r in regions], axis=1)   # [T, R]
        out = np.einsum("pr,rcp->cp", e[t_of], G)
    nrm = np.linalg.norm(out)
    sigma = nrm / (snr * np.sqrt(2.0 * out.size)) if nrm > 0 else 0.0
    noise = rng.standard_normal(out.shape) + 1j * rng.standard_normal(out.shape)
    return (out + sigma * noise).astype(np.complex64)


# ---------------------------------------------------------------------------
# Whole workloads
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class SliceSet:
    """One shape class: shared masks, per-slice coil maps and samples."""
    ny: int
    nz: int
    ncoils: int
    masks: np.ndarray            # uint8 [T, ny, nz]
    sens: np.ndarray             # complex64 [S, C, ny, nz]
    ksp: np.ndarray              # complex64 [S, C, P_tot]
    slice_index: np.ndarray      # readout positions of the slices in their volume

    @property
    def nslices(self):
        return self.sens.shape[0]


def _shared_empty(shape, dtype):
    """Zeroed array in an anonymous shared mapping (visible to forked workers)."""
    nbytes = int(np.prod(shape)) * np.dtype(dtype).itemsize
    buf = mmap.mmap(-1, max(nbytes, 1))
    return np.frombuffer(buf, dtype=dtype, count=int(np.prod(shape))).reshape(shape)


_JOB = {}


def _slice_job(i):
    j = _JOB
    ix = int(j["slices"][i])
    if j["dims"] == 3:
        lab = labels_3d_slice(j["ells"], j["nx"], ix, j["ny"], j["nz"])
        s2 = coils_3d_slice(j["C"], j["nx"], ix, j["ny"], j["nz"])
    else:
        lab, s2 = j["lab"], j["s2"]
    rng = np.random.default_rng([j["seed"], 2, ix])
    j["sens"][i] = s2
    j["ksp"][i] = acquire(lab, j["pd"], j["t2"], s2, j["masks"], j["snr"], rng, locs=j["locs"])
    return i


def _class_slices(cfg, cl, slices, workers=None):
    seed = cl.get("seed", cfg["seed"])
    T = cfg["T"]
    ny, nz, C = cl["ny"], cl["nz"], cl["ncoils"]
    masks = vd_poisson_masks(seed, T, ny, nz, cfg["frac"], cfg["center_frac"])
    locs = sample_locations(masks)
    ptot = locs[0].size
    nx = cl["nx"]
    if slices is None:
        if cl["nslices"] == nx:
            slices = np.arange(nx)
        else:                                   # evenly spaced inside the central half
            slices = np.round(np.linspace(nx // 4, 3 * nx // 4 - 1, cl["nslices"])).astype(int)
    slices = np.asarray(slices, dtype=int)
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    workers = max(1, min(workers, len(slices) // 4))
    alloc = _shared_empty if workers > 1 else np.zeros
    sens = alloc((len(slices), C, ny, nz), np.complex64)
    ksp = alloc((len(slices), C, ptot), np.complex64)
    vrng = np.random.default_rng([seed, 1])
    job = dict(dims=cfg["dims"], ny=ny, nz=nz, nx=nx, C=C, seed=seed, masks=masks, locs=locs, snr=cfg["snr"],
               sens=sens, ksp=ksp, slices=slices)
    if cfg["dims"] == 2:
        ells = draw_ellipses(vrng)
        job["lab"] = labels_2d(ells, ny, nz)
        job["s2"] = coils_2d(C, ny, nz)
    else:
        ells = draw_ellipsoids(vrng)
    job["ells"] = ells
    job["pd"] = np.array([e["pd"] for e in ells])
    job["t2"] = np.array([e["t2"] for e in ells])
    _JOB.clear()
    _JOB.update(job)
    if workers > 1:
        # forked workers write their slices straight into the shared arrays; every slice
        # depends only on (seed, slice index), so the result does not depend on `workers`
        with mp.get_context("fork").Pool(workers) as pool:
            for _ in pool.imap_unordered(_slice_job, range(len(slices)), chunksize=2):
                pass
    else:
        for i in range(len(slices)):
            _slice_job(i)
    _JOB.clear()
    return SliceSet(ny, nz, C, masks, sens, ksp, slices)


def make_config(name: str, slices=None, max_slices=None, workers=None):
    """Generate the workload called ``name`` (a key of CONFIGS).  ``slices`` selects
    readout positions (single class workloads); ``max_slices`` keeps the first n of
    each class."""
    if name not in CONFIGS:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(CONFIGS)}")
    cfg = dict(CONFIGS[name])
    phi = basis(cfg["T"], cfg["K"])
    classes = []
    for cl in cfg["classes"]:
        sel = slices
        if sel is None and max_slices is not None:
            nx = cl["nx"]
            if cl["nslices"] == nx:
                sel = np.arange(nx)[:max_slices]
            else:
                sel = np.round(np.linspace(nx // 4, 3 * nx // 4 - 1, cl["nslices"])).astype(int)[:max_slices]
        classes.append(_class_slices(cfg, cl, sel, workers))
    return dict(cfg=cfg, phi=phi, classes=classes)


def _mask_job(args):
    seed, T, ny, nz, frac = args
    return vd_poisson_masks(seed, T, ny, nz, frac, 0.10)


def training_masks(seed, mask_sets=40, ny=256, nz=256, T=80, frac=0.015, workers=None):
    """The mask sets of the training workload (set m drawn with seed `seed * 1000 + m`)."""
    workers = workers or min(16, os.cpu_count() or 1)
    jobs = [(seed * 1000 + m, T, ny, nz, frac) for m in range(mask_sets)]
    if workers > 1 and mask_sets > 1:
        with mp.get_context("fork").Pool(min(workers, mask_sets)) as pool:
            return np.stack(pool.map(_mask_job, jobs))
    return np.stack([_mask_job(j) for j in jobs])


def _train_job(i):
    j = _JOB
    g = j["first"] + i
    rng = np.random.default_rng([j["seed"], 3, g])
    ells = draw_ellipses(rng)
    lab = labels_2d(ells, j["ny"], j["nz"])
    s2 = coils_2d(j["C"], j["ny"], j["nz"], rot=rng.uniform(0, 2 * np.pi))
    m = g % j["mask_sets"]
    pd = np.array([e["pd"] for e in ells])
    t2 = np.array([e["t2"] for e in ells])
    j["sens"][i] = s2
    y = acquire(lab, pd, t2, s2, j["masks"][m], rng.uniform(*j["snr_range"]), rng, locs=j["locs"][m])
    j["ksp"][i, :, :y.shape[1]] = y
    return i


def make_training_chunk(first, n, seed, masks, C=8, snr_range=(15.0, 40.0), workers=None):
    """Training slices [first, first + n): independent 2D phantoms (slice g uses mask set
    g mod len(masks), coil ring rotated at random, SNR ~ U(snr_range)).  Returns
    (sens [n, C, ny, nz], ksp [n, C, Pmax] zero padded, ptot [n], mask_id [n])."""
    mask_sets, T, ny, nz = masks.shape
    locs = [sample_locations(masks[m]) for m in range(mask_sets)]
    ptot = np.array([locs[(first + i) % mask_sets][0].size for i in range(n)])
    pmax = int(max(l[0].size for l in locs))
    workers = max(1, min(workers or min(16, os.cpu_count() or 1), n // 4))
    alloc = _shared_empty if workers > 1 else np.zeros
    sens = alloc((n, C, ny, nz), np.complex64)
    ksp = alloc((n, C, pmax), np.complex64)
    _JOB.clear()
    _JOB.update(first=first, seed=seed, ny=ny, nz=nz, C=C, mask_sets=mask_sets, masks=masks, locs=locs,
                snr_range=snr_range, sens=sens, ksp=ksp)
    if workers > 1:
        with mp.get_context("fork").Pool(workers) as pool:
            for _ in pool.imap_unordered(_train_job, range(n), chunksize=4):
                pass
    else:
        for i in range(n):
            _train_job(i)
    _JOB.clear()
    return sens, ksp, ptot, (first + np.arange(n)) % mask_sets


def make_training_slices(n, seed, mask_sets=40, ny=256, nz=256, C=8, T=80, K=4, frac=0.015,
                         snr_range=(15.0, 40.0), first=0):
    """Independent 2D training slices (random phantom, coil rotation, SNR); slice i uses
    mask set i % mask_sets.  Returns (phi, masks [mask_sets,T,ny,nz], sens [n,C,ny,nz],
    ksp list of [C,P_i] arrays, mask_id [n])."""
    phi = basis(T, K)
    masks = np.stack([vd_poisson_masks(seed * 1000 + m, T, ny, nz, frac, 0.10) for m in range(mask_sets)])
    locs = [sample_locations(masks[m]) for m in range(mask_sets)]
    sens = np.empty((n, C, ny, nz), dtype=np.complex64)
    ksp, mid = [], np.empty(n, dtype=np.int64)
    for i in range(n):
        g = first + i
        rng = np.random.default_rng([seed, 3, g])
        ells = draw_ellipses(rng)
        lab = labels_2d(ells, ny, nz)
        s2 = coils_2d(C, ny, nz, rot=rng.uniform(0, 2 * np.pi))
        m = g % mask_sets
        pd = np.array([e["pd"] for e in ells])
        t2 = np.array([e["t2"] for e in ells])
        sens[i] = s2
        ksp.append(acquire(lab, pd, t2, s2, masks[m], rng.uniform(*snr_range), rng, locs=locs[m]))
        mid[i] = m
    return phi, masks, sens, ksp, mid
