"""Variant space, genome encoding and features.

A variant is (tile per axis, staging, RK-stage fusion, waves-per-EU hint).
Staging: 0 = each cell reads its stencil from global memory, 1 = LDS tiles,
2 = register march (a wave per 64-column strip, x-neighbours through DPP lane
shifts; tile[0] is then 64; 2D: tile[1] rows per wave marching along y; 3D:
tile[1] rows = waves per block marching along z, fused or one stage).  The genome is its bit string: 2 bits per active axis for
the tile (8, 16, 32, 64), 2 bits for staging, 1 bit for fusion, 2 bits for
the hint (0 = compiler's choice, 3, 4, 5).  The paper's genome encodes Manifest /
Delayed choices and launch configurations of generated code ("Tuning
Targets"); here LDS staging and stage fusion are the storage-versus-recompute
choices and tile and occupancy hint are the launch configuration.

An optional axis adds the paper's own Manifest points to the LDS family
("Annotating By Hand"): an LDS tile keeps face fluxes (manifest 0), face
states with each cell solving both its faces (1), or both (2); keys of
manifest 1 and 2 end in "_m1" / "_m2".  It is outside the genome: the
search strategies run on the base space, the databases and the component
attribution (`analysis.py`) see it.
"""
from __future__ import annotations

import itertools
import math

TILE_VALUES = (8, 16, 32, 64)
MARCH3D_ROWS = (4, 8, 12, 16)   # rows (= waves) per block of the 3D register march: 4, 8 one stage;
                                # 8, 12 fused (stage-1 rows; 16 exceeds the LDS)
WAVE_VALUES = (0, 3, 4, 5)
KMAXR = 8                  # cells per thread the LDS kernels keep in registers
MAX_LDS_BYTES = 160 * 1024  # per workgroup on gfx950
STATIC_LDS = 16 * 8 + 64


def threads_for(variant: dict, ndim: int) -> int:
    """Workgroup size: 256, or 512 when an LDS tile needs more than KMAXR cells per thread;
    the 3D register march runs one wave per tile row."""
    if variant["lds"] == 2 and ndim == 3:
        return 64 * variant["tile"][1]
    if variant["lds"] != 1:
        return 256
    c1 = region(variant, ndim, 2 if variant["fuse"] else 0)
    tile = region(variant, ndim, 0)
    for t in (256, 512):
        if max(c1, tile) <= KMAXR * t:
            return t
    return 512


def region(variant: dict, ndim: int, halo: int) -> int:
    n = 1
    for a in range(ndim):
        n *= variant["tile"][a] + 2 * halo
    return n


def lds_bytes(variant: dict, ndim: int, esize: int) -> int:
    """Dynamic LDS of the LDS kernels: primitive region plus the largest face-flux block,
    plus lower and upper face values of the primitive region when face states are kept."""
    t = list(variant["tile"][:ndim])
    H = 4 if variant["fuse"] else 2
    vin = 1
    for a in range(ndim):
        vin *= t[a] + 2 * H
    c1 = [x + 4 for x in t] if variant["fuse"] else t
    fmax = 0
    for a in range(ndim):
        f1 = 1
        f2 = 1
        for b in range(ndim):
            f1 *= c1[b] + (1 if b == a else 0)
            f2 *= t[b] + (1 if b == a else 0)
        fmax = max(fmax, f1, f2)
    kept = 2 * vin if variant.get("manifest", 0) else 0
    return esize * (ndim + 2) * (vin + fmax + kept)


def march3d_fused_lds(rows: int, esize: int) -> int:
    """Dynamic LDS of the fused 3D march: two primitive planes of rows + 4 and rows
    rows, two 3-slot y-flux rings of rows + 1 and rows - 3 faces, 5 fields x 64 lanes."""
    return esize * 5 * 64 * (2 * (rows + 4) + 2 * rows + 3 * (rows + 1) + 3 * (rows - 3))


def statically_valid(variant: dict, ndim: int, esize: int) -> bool:
    if variant["lds"] == 2:
        if ndim == 2:
            return variant["tile"][0] == 64
        if ndim != 3 or variant["tile"][0] != 64:
            return False
        rows = variant["tile"][1]
        if not variant["fuse"]:
            return rows in (4, 8)
        return 6 <= rows <= 12 and march3d_fused_lds(rows, esize) + STATIC_LDS <= MAX_LDS_BYTES
    if not variant["lds"]:
        return True
    if lds_bytes(variant, ndim, esize) + STATIC_LDS > MAX_LDS_BYTES:
        return False
    c1 = region(variant, ndim, 2 if variant["fuse"] else 0)
    return max(c1, region(variant, ndim, 0)) <= KMAXR * threads_for(variant, ndim)


def make_variant(tile, lds, fuse, waves, ndim, manifest: int = 0) -> dict:
    t = tuple(tile) + (1,) * (3 - len(tile))
    if lds == 2:
        t = (64,) + t[1:]
    v = {"tile": t, "lds": int(lds), "fuse": int(fuse), "waves_per_eu": int(waves)}
    if manifest and lds == 1:
        v["manifest"] = int(manifest)
    v["threads"] = threads_for(v, ndim)
    return v


def enumerate_space(ndim: int, manifest: bool = False) -> list:
    out = []
    for tile in itertools.product(TILE_VALUES, repeat=ndim):
        for lds in (0, 1):
            for fuse in (0, 1):
                for w in WAVE_VALUES:
                    out.append(make_variant(tile, lds, fuse, w, ndim))
                    if manifest and lds == 1:
                        out += [make_variant(tile, lds, fuse, w, ndim, m) for m in (1, 2)]
    if ndim == 2:
        for rows in TILE_VALUES:
            for fuse in (0, 1):
                for w in WAVE_VALUES:
                    out.append(make_variant((64, rows), 2, fuse, w, ndim))
    if ndim == 3:
        for rows in MARCH3D_ROWS:
            for planes in TILE_VALUES:
                for fuse in (0, 1):
                    for w in WAVE_VALUES:
                        out.append(make_variant((64, rows, planes), 2, fuse, w, ndim))
    return out


def key(variant: dict) -> str:
    t = variant["tile"]
    k = f"t{t[0]}x{t[1]}x{t[2]}_l{variant['lds']}_f{variant['fuse']}_w{variant['waves_per_eu']}"
    m = variant.get("manifest", 0)
    return k + (f"_m{m}" if m else "")


# ---- genome -------------------------------------------------------------------------------

def genome_bits(ndim: int) -> int:
    return 2 * ndim + 5


def _axis_values(lds: int, ndim: int, a: int):
    return MARCH3D_ROWS if (lds == 2 and ndim == 3 and a == 1) else TILE_VALUES


def encode(variant: dict, ndim: int) -> str:
    bits = []
    for a in range(ndim):
        i = _axis_values(variant["lds"], ndim, a).index(variant["tile"][a])
        bits += [(i >> 1) & 1, i & 1]
    bits += [(variant["lds"] >> 1) & 1, variant["lds"] & 1, variant["fuse"]]
    w = WAVE_VALUES.index(variant["waves_per_eu"])
    bits += [(w >> 1) & 1, w & 1]
    return "".join(str(b) for b in bits)


def decode(genome: str, ndim: int) -> dict:
    b = [int(c) for c in genome]
    if len(b) != genome_bits(ndim):
        raise ValueError("genome length")
    o = 2 * ndim
    lds = b[o] * 2 + b[o + 1]
    tile = [_axis_values(lds, ndim, a)[b[2 * a] * 2 + b[2 * a + 1]] for a in range(ndim)]
    return make_variant(tile, lds, b[o + 2], WAVE_VALUES[b[o + 3] * 2 + b[o + 4]], ndim)


# ---- features of the cost model ---------------------------------------------------------

def features(variant: dict, ndim: int, esize: int) -> list:
    t = variant["tile"]
    cells = region(variant, ndim, 0)
    halo = region(variant, ndim, 2 if variant["fuse"] else 0) / cells
    loads = region(variant, ndim, 4 if variant["fuse"] else 2) / cells
    w = variant["waves_per_eu"]
    f = [math.log2(t[a]) / 6.0 for a in range(3)]
    f += [1.0 if variant["lds"] == k else 0.0 for k in (0, 1, 2)]
    f += [float(variant["fuse"]), float((variant["lds"] > 0) * variant["fuse"])]
    f += [1.0 if w == x else 0.0 for x in WAVE_VALUES]
    f += [math.log2(cells) / 18.0, halo / 4.0, math.log2(loads) / 4.0,
          lds_bytes(variant, ndim, esize) / MAX_LDS_BYTES if variant["lds"] == 1 else 0.0,
          variant["threads"] / 512.0]
    return f


N_FEATURES = 18
