"""Test helpers: oracle objects and DoF matching by exact position codes."""
import functools

import numpy as np

import synth
from oracle import octree
from oracle.hierarchy import Hierarchy, level_pairs
from oracle.space import Space


def perm_from_codes(codes_ref, codes_other):
    """perm such that other[perm[i]] is the DoF with reference code i."""
    pos = {tuple(c): i for i, c in enumerate(np.asarray(codes_other).tolist())}
    return np.array([pos[tuple(c)] for c in np.asarray(codes_ref).tolist()], dtype=np.int64)


@functools.lru_cache(maxsize=None)
def oracle_tree(name):
    return octree.build_mesh(DESCS[name])


@functools.lru_cache(maxsize=None)
def oracle_hierarchy(name, k, scheme="h"):
    return Hierarchy(oracle_tree(name), k, scheme)


DESCS = {
    "tiny": synth.CFG1_TINY,
    "small": synth.small_mesh(),
    "cfg1": synth.CFG1,
    "small_m1": synth.ball_mesh("small_m1", 2, 0, 2, r=0.7, centre=(-0.4, -0.3, -0.5), lo=-1.0, hi=1.0),
    # the sphere-cut refinement of the p-multigrid workload on a 2^3 coarse grid
    "spheres_small": synth.mesh_desc("cube2_spheres2", 2, -1.0, 1.0, 0,
                                     [(synth.SPHERE_CUT, (0.0, 0.0, 0.0, 0.3, 0.7))] * 2),
}

SCHEME_CODES = {"h": 0, "p_then_h": 1, "h_then_p": 2, "hp": 5}
