"""Seeded synthetic face batches for tests and benchmarks.

This module holds no transfer arithmetic: it only places hanging faces in the
unit cube, fills both face buffers with a smooth field sampled at the cell
centres, and lays out the per-face descriptors.  The test oracle and the HIP
library both consume what it produces; neither is imported here.

Buffer convention (the library's header states the same contract): a face
whose normal is axis a = o mod 3 stores 2k x p x p cells, axis 0 fastest and
the unknowns of a cell innermost; normal index [0, k) is the - side; the fine
patch is on the + side for o < 3.  Fine subface s = sb + 3 sc covers fine
columns [sb p, (sb + 1) p) x [sc p, (sc + 1) p) of the coarse face.

Workloads (all seeds are 15814 + workload number; draw order is fixed below):

1  64 faces, p = 9, k = 3, U = 1; o = f mod 6, s = (f div 6) mod 9; a random
   cubic plus sin(kappa . x), kappa_i ~ U[0.5, 2].
2  20,000 faces, p = 9, k = 3, U = 59; o, s uniform; per unknown 8 Gaussian
   bumps (amplitude N(0,1), centre U[0,1]^3, width U[0.2, 1]) plus
   N(0, 1e-3^2) noise on every stored value.
3  workload 2 with unknown u (field and noise) scaled by 10^(-6 + 9 u / 58).
4  50,000 faces: p in {6, 9, 12} at 30/50/20 %, k in {2, 3}, scheme and
   direction uniform, U = 59, fields as workload 2.
5  three seeded 3-level AMR meshes (see workload5).
6  hanging faces between patches with halos (see patch_transitions): 6,003
   fine patches of 9^3 cells, nine per coarse face, k = 3, U = 59.
7  two-dimensional faces (see faces_2d): 200,000 faces, p = 9, k = 3, U = 59.
8  the transition zone of one seeded mesh as one pool of patches (see
   mesh_patches): 34,481 patches, 39,942 hanging faces, k = 3, U = 59.
Faces sit on a grid of 9^3 coarse patches (h_c = 1/81, h_f = 1/243).
"""

from dataclasses import dataclass, field

import numpy as np
import torch

SEED_BASE = 15814
H_FINE = 1.0 / 243.0


@dataclass
class FaceBatch:
    """Independent hanging faces sharing (p, k, U).  Every face owns one coarse
    and one fine buffer of 2k p^2 U elements inside the flat `coarse` and
    `fine` tensors, at the element offsets given per face."""

    p: int
    k: int
    U: int
    orientation: torch.Tensor  # int8 [n]
    subface: torch.Tensor  # int8 [n]
    coarse_offset: torch.Tensor  # int64 [n]
    fine_offset: torch.Tensor  # int64 [n]
    coarse: torch.Tensor  # float [n * 2k p^2 U]
    fine: torch.Tensor  # float [n * 2k p^2 U]
    origin: torch.Tensor = field(default=None)  # float64 [n, 3] physical corner

    @property
    def n(self):
        return int(self.orientation.numel())

    @property
    def face_elems(self):
        return 2 * self.k * self.p * self.p * self.U

    def to(self, device):
        kw = {}
        for name in ("orientation", "subface", "coarse_offset", "fine_offset", "coarse", "fine", "origin"):
            v = getattr(self, name)
            kw[name] = None if v is None else v.to(device)
        return FaceBatch(self.p, self.k, self.U, **kw)


# ---------------------------------------------------------------------------
# Cell centres of a face buffer, in fine-mesh units relative to the face
# (face plane at normal coordinate 0, coarse face lower corner at 0).
# ---------------------------------------------------------------------------
def _grid(o, p, k, device):
    a = o % 3
    ext = [p, p, p]
    ext[a] = 2 * k
    i2, i1, i0 = torch.meshgrid(
        torch.arange(ext[2], device=device),
        torch.arange(ext[1], device=device),
        torch.arange(ext[0], device=device),
        indexing="ij",
    )
    return a, torch.stack([i0.reshape(-1), i1.reshape(-1), i2.reshape(-1)], dim=1).to(torch.float64)


def coarse_centres(o, p, k, device="cpu"):
    a, idx = _grid(o, p, k, device)
    pos = 3.0 * idx + 1.5
    pos[:, a] = 3.0 * (idx[:, a] - k) + 1.5
    return pos


def fine_centres(o, p, k, s, device="cpu"):
    a, idx = _grid(o, p, k, device)
    b, c = [ax for ax in range(3) if ax != a]
    pos = idx + 0.5
    pos[:, a] = idx[:, a] - k + 0.5
    pos[:, b] += (s % 3) * p
    pos[:, c] += (s // 3) * p
    return pos


# ---------------------------------------------------------------------------
# Smooth fields
# ---------------------------------------------------------------------------
@dataclass
class BumpField:
    """Sum of Gaussian bumps per unknown: amp [U, B], centre [U, B, 3],
    width [U, B]; optional per-unknown scale [U]."""

    amp: torch.Tensor
    centre: torch.Tensor
    width: torch.Tensor
    scale: torch.Tensor = None

    def __call__(self, x):
        """x: [N, 3] physical positions -> [N, U] values (float64)."""
        U, B = self.amp.shape
        dev = x.device
        out = torch.zeros(x.shape[0], U, dtype=torch.float64, device=dev)
        amp, cen, wid = self.amp.to(dev), self.centre.to(dev), self.width.to(dev)
        for j in range(B):
            d2 = ((x[:, None, :] - cen[None, :, j, :]) ** 2).sum(-1)  # [N, U]
            out += amp[None, :, j] * torch.exp(-d2 / (2.0 * wid[None, :, j] ** 2))
        if self.scale is not None:
            out *= self.scale.to(dev)[None, :]
        return out


@dataclass
class CubicSineField:
    """sum_{|alpha|<=3} a_alpha (x - 1/2)^alpha + sin(kappa . x), one unknown."""

    coeffs: torch.Tensor  # [20]
    kappa: torch.Tensor  # [3]

    def __call__(self, x):
        y = x - 0.5
        out = torch.sin(x @ self.kappa.to(x.device))
        i = 0
        for t in range(4):
            for e0 in range(t + 1):
                for e1 in range(t + 1 - e0):
                    e2 = t - e0 - e1
                    out = out + self.coeffs[i].item() * y[:, 0] ** e0 * y[:, 1] ** e1 * y[:, 2] ** e2
                    i += 1
        return out[:, None]


def bump_field(gen, U, n_bumps=8, scaled=False):
    amp = torch.randn(U, n_bumps, generator=gen, dtype=torch.float64)
    centre = torch.rand(U, n_bumps, 3, generator=gen, dtype=torch.float64)
    width = 0.2 + 0.8 * torch.rand(U, n_bumps, generator=gen, dtype=torch.float64)
    scale = None
    if scaled:
        u = torch.arange(U, dtype=torch.float64)
        scale = 10.0 ** (-6.0 + 9.0 * u / max(U - 1, 1))
    return BumpField(amp, centre, width, scale)


def cubic_sine_field(gen):
    coeffs = torch.randn(20, generator=gen, dtype=torch.float64)
    kappa = 0.5 + 1.5 * torch.rand(3, generator=gen, dtype=torch.float64)
    return CubicSineField(coeffs, kappa)


# ---------------------------------------------------------------------------
# Face placement and buffer filling
# ---------------------------------------------------------------------------
def face_origins(gen, orientation, p):
    """Physical position of each coarse face's corner: the face plane sits on an
    interior patch boundary of a 9^3 patch grid and the face covers one patch
    side (p coarse cells of width 1/81 when p = 9)."""
    n = orientation.numel()
    cell = torch.randint(1, 8, (n, 3), generator=gen).to(torch.float64) / 9.0
    return cell


def fill_buffers(batch, field_fn, noise_sigma=0.0, gen=None, chunk=2048, noise_scale=None):
    """Sample field_fn at every cell centre of every face (both buffers), add
    iid N(0, noise_sigma^2) noise (times noise_scale[u] per unknown if given),
    and store into batch.coarse / batch.fine."""
    p, k, U = batch.p, batch.k, batch.U
    dev = batch.coarse.device
    ncell = 2 * k * p * p
    E = ncell * U
    cc = {o: coarse_centres(o, p, k, dev) for o in range(6)}
    fc = {(o, s): fine_centres(o, p, k, s, dev) for o in range(6) for s in range(9)}
    orient = batch.orientation.cpu().tolist()
    sub = batch.subface.cpu().tolist()
    origin = batch.origin.to(dev)
    cview = batch.coarse.view(-1)
    fview = batch.fine.view(-1)
    coff = batch.coarse_offset.cpu().tolist()
    foff = batch.fine_offset.cpu().tolist()
    contiguous = coff == [f * E for f in range(batch.n)] and foff == coff
    noise_gen = None
    if noise_sigma:
        seed = int(torch.randint(0, 2**62, (1,), generator=gen).item())
        noise_gen = torch.Generator(device=dev).manual_seed(seed)
    for f0 in range(0, batch.n, chunk):
        f1 = min(batch.n, f0 + chunk)
        pos_c = torch.stack([cc[orient[f]] for f in range(f0, f1)]) * H_FINE + origin[f0:f1, None, :]
        pos_f = torch.stack([fc[(orient[f], sub[f])] for f in range(f0, f1)]) * H_FINE + origin[f0:f1, None, :]
        vc = field_fn(pos_c.reshape(-1, 3)).reshape(f1 - f0, E)
        vf = field_fn(pos_f.reshape(-1, 3)).reshape(f1 - f0, E)
        if noise_sigma:
            nc = noise_sigma * torch.randn(vc.shape, generator=noise_gen, dtype=torch.float64, device=dev)
            nf_ = noise_sigma * torch.randn(vf.shape, generator=noise_gen, dtype=torch.float64, device=dev)
            if noise_scale is not None:
                sc = noise_scale.to(dev).repeat(ncell)[None, :]
                nc *= sc
                nf_ *= sc
            vc += nc
            vf += nf_
        if contiguous:
            cview[f0 * E : f1 * E] = vc.reshape(-1).to(cview.dtype)
            fview[f0 * E : f1 * E] = vf.reshape(-1).to(fview.dtype)
        else:
            for i, f in enumerate(range(f0, f1)):
                cview[coff[f] : coff[f] + E] = vc[i].to(cview.dtype)
                fview[foff[f] : foff[f] + E] = vf[i].to(fview.dtype)


def _contiguous_batch(orientation, subface, p, k, U, dtype, device, origin):
    n = orientation.numel()
    elems = 2 * k * p * p * U
    offs = torch.arange(n, dtype=torch.int64) * elems
    return FaceBatch(
        p, k, U,
        orientation.to(torch.int8).to(device),
        subface.to(torch.int8).to(device),
        offs.to(device),
        offs.clone().to(device),
        torch.zeros(n * elems, dtype=dtype, device=device),
        torch.zeros(n * elems, dtype=dtype, device=device),
        origin,
    )


def workload1(device="cpu", dtype=torch.float64):
    """64 faces, p = 9, k = 3, U = 1, every (orientation, subface) pair present."""
    gen = torch.Generator().manual_seed(SEED_BASE + 1)
    f = torch.arange(64)
    orient, sub = f % 6, (f // 6) % 9
    origin = face_origins(gen, orient, 9)
    batch = _contiguous_batch(orient, sub, 9, 3, 1, dtype, device, origin)
    fill_buffers(batch, cubic_sine_field(gen))
    return batch


def pair_faces(n, p, k, U, seed, device="cpu", dtype=torch.float64):
    """n faces with o = f mod 6 and s = (f div 6) mod 9 (every orientation /
    subface pair once n >= 54), bump fields plus 1e-3 noise."""
    gen = torch.Generator().manual_seed(seed)
    f = torch.arange(n)
    orient, sub = f % 6, (f // 6) % 9
    origin = face_origins(gen, orient, p)
    fieldfn = bump_field(gen, U)
    batch = _contiguous_batch(orient, sub, p, k, U, dtype, device, origin)
    fill_buffers(batch, fieldfn, noise_sigma=1e-3, gen=gen, noise_scale=fieldfn.scale)
    return batch


def uniform_faces(n, p, k, U, seed, device="cpu", dtype=torch.float64, scaled=False, noise=1e-3):
    """n faces with uniform orientation and subface, bump fields plus noise."""
    gen = torch.Generator().manual_seed(seed)
    orient = torch.randint(0, 6, (n,), generator=gen)
    sub = torch.randint(0, 9, (n,), generator=gen)
    origin = face_origins(gen, orient, p)
    fieldfn = bump_field(gen, U, scaled=scaled)
    batch = _contiguous_batch(orient, sub, p, k, U, dtype, device, origin)
    fill_buffers(batch, fieldfn, noise_sigma=noise, gen=gen, noise_scale=fieldfn.scale)
    return batch


def workload2(n_faces=20000, device="cpu", dtype=torch.float64, U=59):
    """20,000 faces, p = 9, k = 3, U = 59 (CCZ4-sized state), bump fields."""
    return uniform_faces(n_faces, 9, 3, U, SEED_BASE + 2, device, dtype)


def workload3(n_faces=20000, device="cpu", dtype=torch.float64, U=59):
    """Workload 2's faces and fields with unknown u scaled by 10^(-6 + 9u/58)
    (magnitudes 1e-6 .. 1e3; the scaling draws no random numbers)."""
    return uniform_faces(n_faces, 9, 3, U, SEED_BASE + 2, device, dtype, scaled=True)


def sentinel_fill_(t, value=-7.25e11):
    """Fill a destination buffer with a recognisable value."""
    t.fill_(value)
    return t


# ---------------------------------------------------------------------------
# Workload 4: an uneven mix of hanging faces in shared pools
# ---------------------------------------------------------------------------
@dataclass
class MixedBatch:
    """Independent hanging faces of different (p, k, scheme, direction) whose
    coarse and fine buffers live in two flat pools.  Face f owns
    2 k_f p_f^2 U elements at coarse_offset[f] / fine_offset[f]."""

    U: int
    p: torch.Tensor  # int64 [n] (host)
    k: torch.Tensor
    scheme: torch.Tensor
    direction: torch.Tensor  # 0 interpolate, 1 restrict
    orientation: torch.Tensor  # int8 [n] (device)
    subface: torch.Tensor
    coarse_offset: torch.Tensor  # int64 [n] (device)
    fine_offset: torch.Tensor
    coarse: torch.Tensor
    fine: torch.Tensor

    @property
    def n(self):
        return int(self.p.numel())

    def groups(self):
        """{(direction, scheme, p, k): host index tensor of its faces}, faces
        in their interleaved pool order."""
        key = ((self.direction * 4 + self.scheme) * 64 + self.p) * 4 + self.k
        out = {}
        for kv in torch.unique(key).tolist():
            idx = torch.nonzero(key == kv).flatten()
            f = int(idx[0])
            out[(int(self.direction[f]), int(self.scheme[f]), int(self.p[f]), int(self.k[f]))] = idx
        return out

    def subset(self, idx):
        """Descriptor arrays (device) of the faces idx (host index tensor)."""
        dev = self.orientation.device
        i = idx.to(dev)
        return (self.orientation[i].contiguous(), self.subface[i].contiguous(),
                self.coarse_offset[i].contiguous(), self.fine_offset[i].contiguous())


def workload4(n_faces=50000, device="cpu", dtype=torch.float32, U=59, seed=SEED_BASE + 4,
              k_values=(2, 3), p_values=(6, 9, 12)):
    """50,000 faces: p in {6, 9, 12} at 30/50/20 %, k in {2, 3} uniform, scheme
    in {d-linear, Taylor-2, Taylor-3} uniform, direction Bernoulli(1/2)
    interleaved; bump fields with 1e-3 noise, U = 59.  Other halo depths can
    be mixed in with k_values (uniform over them); faces drawn with k = 1
    use the d-linear scheme, the only one defined there.  p_values replaces
    the three patch sizes (same 30/50/20 % split)."""
    gen = torch.Generator().manual_seed(seed)
    r = torch.rand(n_faces, generator=gen)
    p0, p1, p2 = p_values
    p = torch.where(r < 0.3, p0, torch.where(r < 0.8, p1, p2)).to(torch.int64)
    if tuple(k_values) == (2, 3):
        k = torch.randint(2, 4, (n_faces,), generator=gen)
    else:
        kv = torch.tensor(k_values, dtype=torch.int64)
        k = kv[torch.randint(0, len(k_values), (n_faces,), generator=gen)]
    scheme = torch.randint(1, 4, (n_faces,), generator=gen)
    scheme = torch.where(k == 1, torch.ones_like(scheme), scheme)
    direction = torch.randint(0, 2, (n_faces,), generator=gen)
    orient = torch.randint(0, 6, (n_faces,), generator=gen)
    sub = torch.randint(0, 9, (n_faces,), generator=gen)
    origin = face_origins(gen, orient, 9)
    fieldfn = bump_field(gen, U)
    elems = 2 * k * p * p * U
    offs = torch.cumsum(elems, 0) - elems
    total = int(elems.sum())
    mb = MixedBatch(U, p, k, scheme, direction, orient.to(torch.int8).to(device), sub.to(torch.int8).to(device),
                    offs.to(device), offs.clone().to(device),
                    torch.zeros(total, dtype=dtype, device=device), torch.zeros(total, dtype=dtype, device=device))
    noise_seed = int(torch.randint(0, 2**62, (1,), generator=gen).item())
    noise_gen = torch.Generator(device=device).manual_seed(noise_seed)
    for pp in p_values:
        for kk in k_values:
            sel = torch.nonzero((p == pp) & (k == kk)).flatten()
            if sel.numel() == 0:
                continue
            E = 2 * kk * pp * pp * U
            cc = {o: coarse_centres(o, pp, kk, device) for o in range(6)}
            fc = {(o, s): fine_centres(o, pp, kk, s, device) for o in range(6) for s in range(9)}
            ol, sl = orient[sel].tolist(), sub[sel].tolist()
            for c0 in range(0, sel.numel(), 1024):
                part = sel[c0:c0 + 1024]
                idx = list(range(c0, c0 + part.numel()))
                org = origin[part].to(device)[:, None, :]
                pos_c = torch.stack([cc[ol[i]] for i in idx]) * H_FINE + org
                pos_f = torch.stack([fc[(ol[i], sl[i])] for i in idx]) * H_FINE + org
                vc = fieldfn(pos_c.reshape(-1, 3)).reshape(part.numel(), E)
                vf = fieldfn(pos_f.reshape(-1, 3)).reshape(part.numel(), E)
                vc += 1e-3 * torch.randn(vc.shape, generator=noise_gen, dtype=torch.float64, device=device)
                vf += 1e-3 * torch.randn(vf.shape, generator=noise_gen, dtype=torch.float64, device=device)
                where = (offs[part].to(device)[:, None] + torch.arange(E, device=device)[None, :]).reshape(-1)
                mb.coarse[where] = vc.reshape(-1).to(dtype)
                mb.fine[where] = vf.reshape(-1).to(dtype)
    return mb


# ---------------------------------------------------------------------------
# Workload 5: hanging faces of synthetic 3-level AMR meshes
# ---------------------------------------------------------------------------
@dataclass
class MeshFaces:
    """Hanging faces of an adaptive Cartesian mesh (three-partitioning, 2:1
    balanced).  Coarse face buffers are shared by the nine fine faces that
    cover them; every fine face owns its buffer."""

    p: int
    k: int
    U: int
    n_coarse: int
    orientation: torch.Tensor  # int8 [n]
    subface: torch.Tensor  # int8 [n]
    coarse_offset: torch.Tensor  # int64 [n]
    fine_offset: torch.Tensor  # int64 [n]
    coarse: torch.Tensor
    fine: torch.Tensor
    levels: dict = field(default_factory=dict)  # leaf count per level
    transitions: dict = field(default_factory=dict)  # hanging faces per fine level

    @property
    def n(self):
        return int(self.orientation.numel())

    @property
    def face_elems(self):
        return 2 * self.k * self.p * self.p * self.U


def amr_leaves(seed, base_level=3, radii=(0.3, 0.1)):
    """Leaves {(level, i, j, l)} of a unit-cube spacetree: every patch of the
    base level is split into 3^3 children if its centre lies within radii[0]
    of either of two centres drawn U[0.3, 0.7]^3, and those children again if
    within radii[1]; then refined further until neighbours differ by at most
    one level (2:1 balance)."""
    gen = np.random.default_rng(seed)
    centres = gen.uniform(0.3, 0.7, size=(2, 3))

    def near(level, idx, r):
        h = 3.0 ** -level
        c = (np.asarray(idx) + 0.5) * h
        return np.min(np.linalg.norm(centres - c, axis=1)) <= r

    n0 = 3 ** base_level
    leaves = set()
    for i in range(n0):
        for j in range(n0):
            for l in range(n0):
                leaves.add((base_level, i, j, l))
    for depth, r in enumerate(radii):
        lvl = base_level + depth
        for leaf in [x for x in leaves if x[0] == lvl and near(lvl, x[1:], r)]:
            leaves.discard(leaf)
            for di in range(3):
                for dj in range(3):
                    for dl in range(3):
                        leaves.add((lvl + 1, 3 * leaf[1] + di, 3 * leaf[2] + dj, 3 * leaf[3] + dl))
    # 2:1 balance: refine any leaf with a face neighbour two or more levels finer.
    changed = True
    while changed:
        changed = False
        for leaf in sorted(leaves, key=lambda x: -x[0]):
            lvl, idx = leaf[0], leaf[1:]
            for ax in range(3):
                for sgn in (-1, 1):
                    nb = list(idx)
                    nb[ax] += sgn
                    if not (0 <= nb[ax] < 3 ** lvl):
                        continue
                    coarse = (lvl - 2, *[v // 9 for v in nb])
                    if coarse in leaves:
                        leaves.discard(coarse)
                        for di in range(3):
                            for dj in range(3):
                                for dl in range(3):
                                    leaves.add((lvl - 1, 3 * coarse[1] + di, 3 * coarse[2] + dj, 3 * coarse[3] + dl))
                        changed = True
    return leaves


def hanging_faces(leaves):
    """[(coarse_leaf, fine_leaf, orientation, subface)] for every fine leaf
    face that touches a leaf one level coarser."""
    out = []
    for leaf in leaves:
        lvl, idx = leaf[0], leaf[1:]
        for ax in range(3):
            for sgn in (-1, 1):
                nb = list(idx)
                nb[ax] += sgn
                if not (0 <= nb[ax] < 3 ** lvl) or (lvl, *nb) in leaves:
                    continue
                parent = (lvl - 1, *[v // 3 for v in nb])
                if parent not in leaves:
                    continue  # finer neighbour: seen from its side
                b, c = [x for x in range(3) if x != ax]
                sb = idx[b] - 3 * parent[1 + b]
                sc = idx[c] - 3 * parent[1 + c]
                # fine patch on the + side of the face when it lies above it
                o = ax if sgn < 0 else ax + 3
                out.append((parent, leaf, o, sb + 3 * sc))
    return out


def workload5(n_meshes=3, p=9, k=3, U=59, device="cpu", dtype=torch.float64, seed=SEED_BASE + 5,
              base_level=3):
    """Hanging faces of n_meshes independently seeded 3-level meshes (base
    level 3: 27^3 patches of p^3 cells), with shared coarse face buffers;
    bump fields sampled at every cell centre of both buffers."""
    gen = torch.Generator().manual_seed(seed)
    fieldfn = bump_field(gen, U)
    coarse_keys, records = {}, []
    levels, transitions = {}, {}
    for m in range(n_meshes):
        leaves = amr_leaves(seed * 7 + m, base_level)
        for lf in leaves:
            levels[lf[0]] = levels.get(lf[0], 0) + 1
        for parent, leaf, o, s in sorted(hanging_faces(leaves)):
            key = (m, parent, o)
            if key not in coarse_keys:
                coarse_keys[key] = len(coarse_keys)
            records.append((coarse_keys[key], m, parent, leaf, o, s))
            transitions[leaf[0]] = transitions.get(leaf[0], 0) + 1
    n = len(records)
    E = 2 * k * p * p * U
    orient = torch.tensor([r[4] for r in records], dtype=torch.int8)
    sub = torch.tensor([r[5] for r in records], dtype=torch.int8)
    coff = torch.tensor([r[0] * E for r in records], dtype=torch.int64)
    foff = torch.arange(n, dtype=torch.int64) * E
    mf = MeshFaces(p, k, U, len(coarse_keys), orient.to(device), sub.to(device), coff.to(device),
                   foff.to(device), torch.zeros(len(coarse_keys) * E, dtype=dtype, device=device),
                   torch.zeros(n * E, dtype=dtype, device=device), levels, transitions)
    # Physical placement: the face plane lies between coarse leaf and fine
    # leaf; the coarse face's lower tangential corner is the coarse leaf's.
    origin = torch.zeros(n, 3, dtype=torch.float64)
    hf = torch.zeros(n, dtype=torch.float64)
    for f, (_, _m, parent, leaf, o, s) in enumerate(records):
        a = o % 3
        hc_patch = 3.0 ** -parent[0]
        hf[f] = 3.0 ** -leaf[0] / p
        org = [parent[1 + ax] * hc_patch for ax in range(3)]
        org[a] = (parent[1 + a] + (1 if o < 3 else 0)) * hc_patch
        origin[f] = torch.tensor(org)
    dev = device
    cc = {o: coarse_centres(o, p, k, dev) for o in range(6)}
    fc = {(o, s): fine_centres(o, p, k, s, dev) for o in range(6) for s in range(9)}
    ol, sl = orient.tolist(), sub.tolist()
    filled = torch.zeros(len(coarse_keys), dtype=torch.bool)
    for f0 in range(0, n, 1024):
        f1 = min(n, f0 + 1024)
        idx = range(f0, f1)
        org = origin[f0:f1].to(dev)[:, None, :]
        h = hf[f0:f1].to(dev)[:, None, None]
        pos_f = torch.stack([fc[(ol[i], sl[i])] for i in idx]) * h + org
        vf = fieldfn(pos_f.reshape(-1, 3)).reshape(f1 - f0, E)
        mf.fine[f0 * E:f1 * E] = vf.reshape(-1).to(dtype)
        # coarse buffers: fill once per coarse face, from its first fine face
        firsts = [i for i in idx if not filled[records[i][0]]]
        for i in firsts:
            filled[records[i][0]] = True
        if firsts:
            sel = torch.tensor(firsts)
            orgc = origin[sel].to(dev)[:, None, :]
            hc = hf[sel].to(dev)[:, None, None]
            pos_c = torch.stack([cc[ol[i]] for i in firsts]) * hc + orgc
            vc = fieldfn(pos_c.reshape(-1, 3)).reshape(len(firsts), E)
            where = (coff[sel].to(dev)[:, None] + torch.arange(E, device=dev)[None, :]).reshape(-1)
            mf.coarse[where] = vc.reshape(-1).to(dtype)
    return mf


@dataclass
class PatchTransitions:
    """Hanging faces between patches (boxes of (p + 2k)^3 cells, interior
    [k, k + p) per axis, axis 0 fastest, unknowns innermost).  Face i joins
    the coarse patch at coarse_offset[i] of `coarse` to the fine patch at
    fine_offset[i] of `fine` (element offsets); fine patches are not shared,
    coarse patches are shared by `faces_per_coarse` faces that sit on one
    coarse face (one orientation, distinct subfaces)."""

    p: int
    k: int
    U: int
    orientation: torch.Tensor
    subface: torch.Tensor
    coarse_offset: torch.Tensor
    fine_offset: torch.Tensor
    coarse: torch.Tensor
    fine: torch.Tensor

    @property
    def n(self):
        return int(self.orientation.numel())

    @property
    def patch_elems(self):
        return (self.p + 2 * self.k) ** 3 * self.U


def patch_transitions(n_faces, p, k, U, seed, device="cpu", dtype=torch.float64, faces_per_coarse=1):
    """Seeded patches for the fused transfer.  Draw order: orientation and
    subface per group (CPU torch generator seeded `seed`), then the coarse
    pool and the fine pool as standard normal values drawn on `device` by a
    generator of that device seeded `seed` (the transfer is linear, so the
    data only need to be finite; every cell of every patch is filled,
    including edge and vertex cells that no call touches)."""
    if faces_per_coarse not in (1, 9):
        raise ValueError("faces_per_coarse must be 1 or 9")
    gen = torch.Generator().manual_seed(seed)
    groups = -(-n_faces // faces_per_coarse)
    o_g = torch.randint(0, 6, (groups,), generator=gen)
    if faces_per_coarse == 9:
        sub = torch.stack([torch.randperm(9, generator=gen) for _ in range(groups)]).reshape(-1)
    else:
        sub = torch.randint(0, 9, (groups,), generator=gen)
    orientation = o_g.repeat_interleave(faces_per_coarse)[:n_faces].to(torch.int8)
    subface = sub[:n_faces].to(torch.int8)
    P3U = (p + 2 * k) ** 3 * U
    coarse_offset = (torch.arange(n_faces) // faces_per_coarse * P3U).to(torch.int64)
    fine_offset = (torch.arange(n_faces) * P3U).to(torch.int64)
    dgen = torch.Generator(device=device).manual_seed(seed)
    coarse = torch.randn(groups * P3U, generator=dgen, dtype=dtype, device=device)
    fine = torch.randn(n_faces * P3U, generator=dgen, dtype=dtype, device=device)
    return PatchTransitions(p, k, U, orientation.to(device), subface.to(device),
                            coarse_offset.to(device), fine_offset.to(device), coarse, fine)


# ---------------------------------------------------------------------------
# Two-dimensional faces
# ---------------------------------------------------------------------------
def faces_2d(n_faces, p, k, U, seed, device="cpu", dtype=torch.float64):
    """Independent two-dimensional hanging faces (buffers of 2k x p cells,
    axis 0 fastest, unknowns innermost), orientation uniform in 0..3 and
    subface in 0..2 (CPU generator seeded `seed`), every stored value standard
    normal (a generator of `device` seeded `seed`).  Returned as a FaceBatch
    whose buffers each hold 2k p U elements."""
    gen = torch.Generator().manual_seed(seed)
    orient = torch.randint(0, 4, (n_faces,), generator=gen).to(torch.int8)
    sub = torch.randint(0, 3, (n_faces,), generator=gen).to(torch.int8)
    elems = 2 * k * p * U
    offs = torch.arange(n_faces, dtype=torch.int64) * elems
    dgen = torch.Generator(device=device).manual_seed(seed)
    coarse = torch.randn(n_faces * elems, generator=dgen, dtype=dtype, device=device)
    fine = torch.randn(n_faces * elems, generator=dgen, dtype=dtype, device=device)
    return FaceBatch(p, k, U, orient.to(device), sub.to(device), offs.to(device), offs.clone().to(device),
                     coarse, fine)


# ---------------------------------------------------------------------------
# Workload 8: the transition zone of a synthetic AMR mesh, as patches
# ---------------------------------------------------------------------------
@dataclass
class MeshPatches:
    """Patches (boxes of (p + 2k)^3 cells with face halos) of the leaves that
    take part in a hanging face of amr_leaves meshes, all in one pool; face i
    joins the coarse leaf at coarse_offset[i] to the fine leaf at
    fine_offset[i] (element offsets into `pool`)."""

    p: int
    k: int
    U: int
    n_patches: int
    orientation: torch.Tensor
    subface: torch.Tensor
    coarse_offset: torch.Tensor
    fine_offset: torch.Tensor
    pool: torch.Tensor

    @property
    def n(self):
        return int(self.orientation.numel())


def mesh_patches(n_meshes=1, p=9, k=3, U=59, device="cpu", dtype=torch.float64, seed=SEED_BASE + 8,
                 base_level=3, chunk=256):
    """The leaves adjacent to a resolution transition of n_meshes seeded
    meshes (amr_leaves), one patch each, filled with bump fields sampled at
    every cell centre of the box (interior and halos: the halos then hold the
    values a halo refresh would produce)."""
    gen = torch.Generator().manual_seed(seed)
    fieldfn = bump_field(gen, U)
    index, faces = {}, []
    for m in range(n_meshes):
        leaves = amr_leaves(seed * 7 + m, base_level)
        for parent, leaf, o, s in sorted(hanging_faces(leaves)):
            for key in ((m, parent), (m, leaf)):
                if key not in index:
                    index[key] = len(index)
            faces.append((index[(m, parent)], index[(m, leaf)], o, s))
    P = p + 2 * k
    P3U = P ** 3 * U
    n_patches = len(index)
    pool = torch.zeros(n_patches * P3U, dtype=dtype, device=device)
    keys = sorted(index, key=index.get)
    g = torch.arange(P, dtype=torch.float64, device=device)
    i2, i1, i0 = torch.meshgrid(g, g, g, indexing="ij")
    local = (torch.stack([i0, i1, i2], dim=-1).reshape(-1, 3) - k + 0.5) / p  # in patch widths
    for c0 in range(0, n_patches, chunk):
        part = keys[c0:c0 + chunk]
        corner = torch.tensor([[leaf[1 + ax] * 3.0 ** -leaf[0] for ax in range(3)] for _, leaf in part],
                              dtype=torch.float64, device=device)
        width = torch.tensor([3.0 ** -leaf[0] for _, leaf in part], dtype=torch.float64, device=device)
        pos = corner[:, None, :] + local[None, :, :] * width[:, None, None]
        vals = fieldfn(pos.reshape(-1, 3)).reshape(len(part), P3U)
        pool[c0 * P3U:(c0 + len(part)) * P3U] = vals.reshape(-1).to(dtype)
    t = torch.tensor(faces, dtype=torch.int64)
    return MeshPatches(p, k, U, n_patches, t[:, 2].to(torch.int8).to(device), t[:, 3].to(torch.int8).to(device),
                       (t[:, 0] * P3U).to(device), (t[:, 1] * P3U).to(device), pool)
