"""Oracle values of sampled particles of a large set, computed one by one.

TEST INFRASTRUCTURE ONLY (tests/ and the benchmark's CPU-baseline leg), like the
oracle itself.

The forward outputs of particle i depend only on particles within a few
smoothing lengths: its force neighbours j (r_ij < max(h_i, h_j)), their and
its own gather neighbours k (r < h), and the gather neighbourhoods that fix
h_k and V_k. The oracle is run on the union of balls around the sampled
particles; a sample is accepted only when every particle on that chain has
its whole gather neighbourhood inside the subset, so its oracle values equal
those of the full set exactly (the oracle's own subset h is self-checking:
a missing neighbour could only make it larger). Balls that fail are widened.
"""
import numpy as np
from scipy.spatial import cKDTree

import oracle


def _dependency_set(tree_sub, xs, h, i):
    """Indices (into the subset) whose h and gather neighbourhoods i depends on."""
    hi = h[i]
    cand = tree_sub.query_ball_point(xs[i], h.max())
    d = xs[cand] - xs[i]
    d -= np.round(d)
    r = np.sqrt((d * d).sum(1))
    cand = np.asarray(cand)
    force = cand[(r < np.maximum(hi, h[cand]))]
    first = np.union1d(force, [i])
    dep = set(first.tolist())
    for j in first:
        dep.update(tree_sub.query_ball_point(xs[j], h[j]))
    return np.fromiter(dep, dtype=np.int64)


def unit_tree(ps):
    """Positions mapped to the unit periodic box and their k-d tree."""
    x = np.mod(ps.x.T, ps.box) / ps.box
    return x, cKDTree(x, boxsize=1.0)


def complete_subsets(ps, samples, params, grow=1.5, max_rounds=6, start=4.0, want=None,
                     max_size=None, tree=None):
    """For sampled indices, balls of the full set on which the oracle's outputs
    at the sample are exact, and those outputs.

    samples are tried in order; with want, the first `want` that complete
    within max_size particles are kept (a candidate deep in a very massive
    clump would need a subset the oracle takes minutes on).
    tree: unit_tree(ps), when the caller has it already.
    Returns (kept samples, list of subset index arrays, dict of sample outputs
    with the samples on the last axis)."""
    x, tree = unit_tree(ps) if tree is None else tree
    k = min(65, ps.n)
    r64 = tree.query(x[samples], k=k)[0][:, k - 1]
    kept, subsets, per = [], [], []
    for s_idx, g in enumerate(samples):
        if want is not None and len(kept) == want:
            break
        radius = start * r64[s_idx]
        for _ in range(max_rounds):
            sub = np.asarray(tree.query_ball_point(x[g], radius), dtype=np.int64)
            if max_size is not None and sub.size > max_size:
                break
            h0 = ps.h[sub]
            if params.h_mode == 1:
                # starting guess only (the root does not depend on it): the
                # distance to the 64th nearest particle, from the positions
                h0 = tree.query(x[sub], k=k)[0][:, k - 1] * ps.box
            o = oracle.forward(ps.x[:, sub], ps.v[:, sub], ps.m[sub], ps.u[sub], h0, params,
                               nbr_mode=1)
            xs = x[sub]
            h = o["h"] / ps.box
            tsub = cKDTree(xs, boxsize=1.0)
            i = int(np.nonzero(sub == g)[0][0])
            dep = _dependency_set(tsub, xs, h, i)
            # complete: the full set has no particle within h_q of q that the subset lacks
            nfull = tree.query_ball_point(xs[dep], h[dep] * (1 + 1e-9), return_length=True)
            nsub = tsub.query_ball_point(xs[dep], h[dep] * (1 + 1e-9), return_length=True)
            if np.all(nfull == nsub):
                kept.append(g)
                subsets.append(sub)
                per.append({key: v[..., i] for key, v in o.items()
                            if isinstance(v, np.ndarray) and v.shape[-1:] == (sub.size,)})
                break
            radius *= grow
        else:
            raise RuntimeError("sampled oracle: sample %d still incomplete" % g)
    if want is not None and len(kept) < want:
        raise RuntimeError("sampled oracle: only %d of %d samples completed" % (len(kept), want))
    out = {key: np.stack([p[key] for p in per], axis=-1) for key in per[0]}
    return np.asarray(kept, dtype=np.int64), subsets, out


def localized_jvp(ps, samples, subsets, params, w_a, w_u, dirs):
    """Oracle directional derivative of L = sum_{i in samples} w_a_i . a_i + w_u_i du_i/dt.

    Every sample's outputs are exact on the union U of its complete subsets,
    and depend on no particle outside U, so the oracle's JVP on U along a
    direction supported on U equals the JVP of the full set. dirs(U) gives
    (dx, dv, du, dalpha, dbeta) on U. Returns (jvp, U, the direction)."""
    U = np.unique(np.concatenate(subsets))
    x = np.mod(ps.x.T, ps.box) / ps.box
    tree = cKDTree(x, boxsize=1.0)
    h0 = ps.h[U]
    if params.h_mode == 1:
        k = min(65, ps.n)
        h0 = tree.query(x[U], k=k)[0][:, k - 1] * ps.box
    d = dirs(U)
    j = oracle.jvp(ps.x[:, U], ps.v[:, U], ps.m[U], ps.u[U], h0, params, *d, nbr_mode=1)
    pos = np.searchsorted(U, samples)
    val = float((w_a * j["d_accel"][:, pos]).sum() + (w_u * j["d_dudt"][pos]).sum())
    return val, U, d


def separated_coordinates_jvp(ps, params, field, w_a, w_u, reach, grid=3, seed=0):
    """Oracle dL/d(coordinate) for grid^3 coordinates of one field ("x", "v" or "u") at once.

    L = sum_i w_a_i . a_i + w_u_i du_i/dt over the whole set. A coordinate of particle p
    moves only the outputs of particles within reach of p (three hops of at most the
    largest h: h and V, then the corrections, density and grad v, then the force pairs).
    The perturbed particles are the ones nearest the points of a grid^3 lattice (randomly
    offset), at least 2 reach apart, so the regions their coordinates move are disjoint:
    one JVP along the sum of their unit directions (components cycling x, y, z) gives each
    derivative as the loss weights contracted with the outputs that moved in its region.
    Checked: the separation, and that every particle whose outputs moved lies within reach
    of its perturbed particle. Returns (particles, components, derivatives)."""
    rng = np.random.default_rng(seed)
    x = np.mod(ps.x.T, ps.box) / ps.box
    tree = cKDTree(x, boxsize=1.0)
    g = (np.stack(np.meshgrid(*[np.arange(grid)] * 3, indexing="ij"), -1).reshape(-1, 3) +
         0.5 + rng.uniform(-0.5, 0.5, 3)) / grid
    parts = tree.query(np.mod(g, 1.0))[1]
    ptree = cKDTree(x[parts], boxsize=1.0)
    sep = ptree.query(x[parts], k=2)[0][:, 1].min()
    assert sep > 2 * reach / ps.box, ("perturbed particles too close", sep, reach)
    comps = np.arange(parts.size) % (1 if field == "u" else 3)
    dx, dv, du = np.zeros_like(ps.x), np.zeros_like(ps.v), np.zeros(ps.n)
    tgt = {"x": dx, "v": dv, "u": du[None]}[field]
    tgt[comps, parts] = 1.0
    j = oracle.jvp(ps.x, ps.v, ps.m, ps.u, ps.h, params, dx, dv, du, 0.0, 0.0, nbr_mode=1)
    contrib = (w_a * j["d_accel"]).sum(0) + w_u * j["d_dudt"]
    moved = np.nonzero((np.abs(j["d_accel"]).sum(0) + np.abs(j["d_dudt"])) > 0)[0]
    owner_d, owner = ptree.query(x[moved])
    assert owner_d.max() < reach / ps.box, ("outputs moved beyond reach", owner_d.max(), reach)
    vals = np.bincount(owner, contrib[moved], minlength=parts.size)
    return parts, comps, vals


def sample_candidates(ps, k, seed):
    """2k candidate samples alternating uniform background and clump particles (the
    clump generator puts the background first)."""
    rng = np.random.default_rng(seed)
    nb = ps.n // 2
    bg = rng.choice(nb, k, replace=False)
    cl = nb + rng.choice(ps.n - nb, k, replace=False)
    return np.stack([bg, cl], axis=1).ravel()


def densest(ps, k, tree=None):
    """The k clump particles with the smallest distance to their 64th neighbour: the
    densest clump cores, where h is smallest and the tree walks go deepest.

    A Plummer sphere's central density is proportional to N / a^3, so with the
    generator's clump table only the 256 particles nearest the centres of the 16
    clumps highest in N / a^3 are ranked; without it every clump particle is."""
    x, tree = unit_tree(ps) if tree is None else tree
    nb = ps.n // 2
    meta = getattr(ps, "meta", {})
    if "clump_centres" in meta:
        cen = np.asarray(meta["clump_centres"], dtype=np.float64)
        cen = np.mod(cen.reshape(-1, 3) if cen.shape[-1] == 3 else cen.T, ps.box) / ps.box
        rank = np.asarray(meta["clump_counts"]) / np.asarray(meta["clump_a"]) ** 3
        top = np.argsort(rank)[::-1][:16]
        near = np.unique(tree.query(cen[top], k=256)[1].ravel())
        cand = near[near >= nb]
    else:
        cand = np.arange(nb, ps.n)
    r64 = tree.query(x[cand], k=65, workers=-1)[0][:, 64]
    return cand[np.argsort(r64)[:k]]


def sampled_oracle(ps, params, k, seed, dense=2, max_size=40000):
    """k samples (each with a complete subset of at most max_size particles) plus the
    `dense` densest core particles (any subset size), their subsets and oracle values."""
    tree = unit_tree(ps)
    kept, subsets, o = complete_subsets(ps, sample_candidates(ps, 4 * k, seed), params,
                                        want=k, max_size=max_size, tree=tree)
    if dense:
        kd, sd, od = complete_subsets(ps, densest(ps, dense, tree), params, tree=tree)
        kept = np.concatenate([kept, kd])
        subsets = subsets + sd
        o = {key: np.concatenate([o[key], od[key]], axis=-1) for key in o}
    return kept, subsets, o
