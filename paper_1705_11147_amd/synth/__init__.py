"""Seeded synthetic read sets for the k-mer analysis workloads.

This module simulates genomes and sequencing reads only.  It holds none of the
k-mer analysis arithmetic (no 2-bit encoding, canonical form, hashing or
counting); the CPU oracle and the GPU path both consume what it produces.

The five workloads follow the shapes of the paper's data sets (section
"Performance Results": a 3.2 Gbp human genome sequenced at about 30x, a
hexaploid wheat genome, 100-250 bp reads) scaled to one GPU.  The recipes are
stated in each function's docstring; the heavy lifting is in ``gen.c``
(SplitMix64 streams, OpenMP), which ``lib()`` compiles with gcc on first use.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_SO = os.path.join(_HERE, "libhmsynth.so")

BASE_SEED = 170511147

_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build_lib(force: bool = False) -> str:
    """Compile gen.c into libhmsynth.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        build_lib()
        L = ctypes.CDLL(_SO)
        L.syn_genome_uniform.argtypes = [_u8p, ctypes.c_int64, ctypes.c_uint64]
        L.syn_genome_uniform.restype = None
        L.syn_diverge.argtypes = [_u8p, _u8p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64]
        L.syn_diverge.restype = None
        L.syn_segmental_repeats.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                            ctypes.c_int64, ctypes.c_uint64]
        L.syn_segmental_repeats.restype = ctypes.c_int64
        L.syn_interspersed_repeats.argtypes = [_u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                               ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64]
        L.syn_interspersed_repeats.restype = ctypes.c_int64
        L.syn_reads.argtypes = [_u8p, _i64p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_uint64, ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int32, ctypes.c_int32, _u8p, _u8p, _i64p, _u8p]
        L.syn_reads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _p8(a: np.ndarray):
    return a.ctypes.data_as(_u8p)


def _p64(a: np.ndarray):
    return a.ctypes.data_as(_i64p)


def seed_for(cfg: int, index: int = 0) -> int:
    """64-bit seed of workload `cfg`, batch/job/set `index` (numpy SeedSequence)."""
    ss = np.random.SeedSequence(BASE_SEED + cfg, spawn_key=(index,))
    return int(ss.generate_state(1, dtype=np.uint64)[0])


def genome_uniform(n: int, seed: int) -> np.ndarray:
    g = np.empty(int(n), dtype=np.uint8)
    lib().syn_genome_uniform(_p8(g), int(n), seed)
    return g


def diverge(src: np.ndarray, rate: float, seed: int, tag: int = 0) -> np.ndarray:
    out = np.empty_like(src)
    lib().syn_diverge(_p8(src), _p8(out), src.size, float(rate), seed, tag)
    return out


def add_segmental_repeats(g: np.ndarray, min_len: int, max_len: int, div: float, target: int, seed: int) -> int:
    return int(lib().syn_segmental_repeats(_p8(g), g.size, min_len, max_len, div, int(target), seed))


def add_interspersed_repeats(g: np.ndarray, n_fam: int, min_len: int, max_len: int, div_lo: float, div_hi: float,
                             target: int, seed: int) -> int:
    return int(lib().syn_interspersed_repeats(_p8(g), g.size, n_fam, min_len, max_len, div_lo, div_hi,
                                              int(target), seed))


def add_satellites(g: np.ndarray, arrays: list[tuple[bytes, float, float]], seed: int) -> int:
    """Overwrite stretches of the genome with tandem satellite arrays: for each
    (motif, fraction of the genome, per-base divergence) one array of that
    length tiles the motif from a random start, with independent substitutions
    at the given rate.  Returns the bases written."""
    rng = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(77,)))
    acgt = np.frombuffer(b"ACGT", np.uint8)
    done = 0
    for motif, frac, div in arrays:
        n = int(frac * g.size)
        if n <= 0:
            continue
        m = np.frombuffer(motif, np.uint8)
        arr = np.resize(m, n).copy()
        hit = rng.random(n) < div
        arr[hit] = acgt[(np.searchsorted(acgt, arr[hit]) + rng.integers(1, 4, int(hit.sum()))) % 4]
        s = int(rng.integers(0, g.size - n))
        g[s:s + n] = arr
        done += n
    return done


@dataclass
class Reads:
    """Fixed-length reads, row-major: ascii[n_reads * read_len], qual likewise
    (numeric Phred, no ASCII offset)."""
    ascii: np.ndarray
    qual: np.ndarray
    n_reads: int
    read_len: int
    start: np.ndarray | None = None
    strand: np.ndarray | None = None

    @property
    def n_bases(self) -> int:
        return self.n_reads * self.read_len

    def offsets(self) -> np.ndarray:
        return np.arange(self.n_reads + 1, dtype=np.int64) * self.read_len


def sample_reads(genome: np.ndarray, chrom_off, L: int, n: int, seed: int, err: float, end_bias: bool = False,
                 r0: int = 0, keep_truth: bool = False, q_mu: float = 32.0, q_sd: float = 6.0, q_min: int = 2,
                 q_max: int = 41) -> Reads:
    """Reads [r0, r0+n) of length L.  Start uniform over the valid starts of
    all chromosomes; reverse complemented with probability 1/2; iid
    substitutions at mean rate `err` (optionally 3x at the read ends); Phred
    iid clamp(rint(N(32, 6)), 2, 41)."""
    chrom_off = np.ascontiguousarray(np.asarray(chrom_off, dtype=np.int64))
    ascii = np.empty(int(n) * L, dtype=np.uint8)
    qual = np.empty(int(n) * L, dtype=np.uint8)
    start = np.empty(int(n), dtype=np.int64) if keep_truth else None
    strand = np.empty(int(n), dtype=np.uint8) if keep_truth else None
    rc = lib().syn_reads(_p8(genome), _p64(chrom_off), chrom_off.size - 1, L, int(r0), int(n), seed, float(err),
                         1 if end_bias else 0, q_mu, q_sd, q_min, q_max, _p8(ascii), _p8(qual),
                         _p64(start) if keep_truth else None, _p8(strand) if keep_truth else None)
    if rc != 0:
        raise ValueError("syn_reads failed (%d): chromosomes shorter than the read length?" % rc)
    return Reads(ascii, qual, int(n), L, start, strand)


@dataclass
class Params:
    """k-mer analysis parameters of a workload."""
    k: int
    qcut: int = 20
    min_depth: int = 2
    ext_min: int = 2
    n_owners: int = 1
    owner: int = 0
    qual_offset: int = 0


@dataclass
class Workload:
    name: str
    params: Params
    genome: np.ndarray
    chrom_off: np.ndarray
    read_len: int
    n_reads: int
    err: float
    end_bias: bool
    seed: int
    meta: dict = field(default_factory=dict)

    def reads(self, r0: int = 0, n: int | None = None, keep_truth: bool = False) -> Reads:
        n = self.n_reads - r0 if n is None else n
        return sample_reads(self.genome, self.chrom_off, self.read_len, n, self.seed, self.err, self.end_bias,
                            r0=r0, keep_truth=keep_truth)

    def size_estimates(self) -> tuple[float, float]:
        """(distinct k-mers, k-mers seen at least twice) expected from this
        recipe: every genome k-mer (all copies), plus about one new k-mer per
        window covering a substitution, of which few repeat."""
        k, L = self.params.k, self.read_len
        W = max(0, L - k + 1)
        per_err = W * min(k, W) / L if L else 0.0  # windows covering an average error position
        errors = self.n_reads * L * self.err
        G = float(self.meta["G"])
        return G + errors * per_err, G * 1.05 + 0.02 * errors * per_err

    @property
    def positions(self) -> int:
        """Valid k-mer positions Sigma_r (L - k + 1) (the generator emits no N bases)."""
        return self.n_reads * max(0, self.read_len - self.params.k + 1)


def tiny(scale: float = 1.0) -> Workload:
    """Plain method, tiny: uniform ACGT genome of 1 Mbp; 200k reads of 100 bp
    at uniform positions, half reverse complemented (20x); 1% iid
    substitutions; Phred clamp(N(32,6),2,41); k=21, Q20, min depth 2."""
    G = max(1000, int(round(1_000_000 * scale)))
    seed = seed_for(0)
    g = genome_uniform(G, seed)
    n = int(round(200_000 * G / 1_000_000))
    return Workload("tiny-1Mbp-20x-k21", Params(k=21), g, np.array([0, G]), 100, n, 0.01, False, seed,
                    {"G": G, "coverage": 20})


def mid(scale: float = 1.0) -> Workload:
    """Plain method, mid: 100 Mbp uniform genome with 5% of it overwritten by
    segmental repeat copies of U[2, 50] kbp at 1% divergence; 30x of 150 bp
    reads (20M reads); 0.5% mean substitution rate, 3x at the read ends;
    k=51, Q20, min depth 2."""
    G = max(60_000, int(round(100_000_000 * scale)))
    seed = seed_for(1)
    g = genome_uniform(G, seed)
    add_segmental_repeats(g, 2000, min(50_000, G // 2), 0.01, int(0.05 * G), seed)
    n = int(round(30 * G / 150))
    return Workload("mid-100Mbp-30x-k51", Params(k=51), g, np.array([0, G]), 150, n, 0.005, True, seed,
                    {"G": G, "coverage": 30})


def mid_heavy(scale: float = 1.0) -> Workload:
    """The mid workload with 2% of the genome replaced by tandem satellite
    arrays, so that a few k-mers hold millions of windows (the heavy hitters
    of section "Parallel k-mer analysis"): a telomere-like (TTAGGG)n and an
    (AATGG)n array at 0.5% each, a poly-A and a (CA)n microsatellite at 0.25%
    each (all 0.2% diverged), and a 171 bp monomer array at 0.5% diverged 1%.
    Same read count, length, errors and k as mid."""
    w = mid(scale)
    rng = np.random.default_rng(np.random.SeedSequence(seed_for(1), spawn_key=(171,)))
    monomer = rng.choice(np.frombuffer(b"ACGT", np.uint8), 171).tobytes()
    add_satellites(w.genome, [(b"TTAGGG", 0.005, 0.002), (b"AATGG", 0.005, 0.002), (b"A", 0.0025, 0.002),
                              (b"CA", 0.0025, 0.002), (monomer, 0.005, 0.01)], seed_for(1))
    w.name = "mid-heavy-100Mbp-30x-k51-2pct-satellite"
    return w


def human_share(scale: float = 1.0, batch_reads: int = 64_000_000) -> Workload:
    """One GPU's share of a human-scale run: 3.2 Gbp genome (uniform ACGT
    plus 45% interspersed repeats: 2000 families of log-uniform consensus
    length in [300, 6000] bp, each copy diverged U(10%, 20%)), 30x of 150 bp
    reads with 0.5% errors, k=51; only k-mers owned by owner 0 of 16 are
    kept; reads come in batches of `batch_reads`."""
    G = max(100_000, int(round(3_200_000_000 * scale)))
    seed = seed_for(2)
    g = genome_uniform(G, seed)
    add_interspersed_repeats(g, 2000, 300, 6000, 0.10, 0.20, int(0.45 * G), seed)
    n = int(round(30 * G / 150))
    return Workload("human-share-3.2Gbp-30x-k51-owner0of16", Params(k=51, n_owners=16, owner=0), g,
                    np.array([0, G]), 150, n, 0.005, False, seed,
                    {"G": G, "coverage": 30, "batch_reads": int(batch_reads * max(scale, 1e-9)) or 1})


def batched_sets(n_sets: int = 64, scale: float = 1.0) -> list[Workload]:
    """Batched: `n_sets` independent read sets; genome sizes
    clip(LogNormal(ln 2 Mbp, ln4/2), 0.5, 8) Mbp, uniform ACGT; coverage
    U(10, 60); 150 bp reads; 1% errors; k=31, Q20, min depth 2."""
    rs = np.random.default_rng(np.random.SeedSequence(BASE_SEED + 3))
    sizes = np.clip(rs.lognormal(math.log(2e6), math.log(4) / 2, n_sets), 0.5e6, 8e6)
    covs = rs.uniform(10, 60, n_sets)
    out = []
    for s in range(n_sets):
        G = max(2000, int(round(sizes[s] * scale)))
        seed = seed_for(3, s)
        g = genome_uniform(G, seed)
        n = int(round(covs[s] * G / 150))
        out.append(Workload("batched-set%02d" % s, Params(k=31), g, np.array([0, G]), 150, n, 0.01, False, seed,
                            {"G": G, "coverage": float(covs[s])}))
    return out


def serving_jobs(n_jobs: int = 200, rate: float = 20.0, scale: float = 1.0) -> tuple[np.ndarray, list]:
    """Serving: Poisson arrivals at `rate` jobs/s; each job is a hexaploid-like
    genome: an ancestor of g ~ log-U[1, 50] Mbp and three homeologous copies,
    each the ancestor with 1.5% iid substitutions (about 3% pairwise), read as
    three chromosomes at 30x of 3g with 150 bp reads, 0.5% errors, k=51.
    Returns (arrival times in seconds, list of job builders); a builder
    returns the job's Workload when called."""
    rs = np.random.default_rng(np.random.SeedSequence(BASE_SEED + 4))
    gaps = rs.exponential(1.0 / rate, n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = np.exp(rs.uniform(math.log(1e6), math.log(50e6), n_jobs))

    def make(j: int) -> Workload:
        g0 = max(1000, int(round(sizes[j] * scale)))
        seed = seed_for(4, j)
        anc = genome_uniform(g0, seed)
        copies = [diverge(anc, 0.015, seed, tag=c + 1) for c in range(3)]
        g = np.concatenate(copies)
        off = np.array([0, g0, 2 * g0, 3 * g0], dtype=np.int64)
        n = int(round(30 * 3 * g0 / 150))
        return Workload("serving-job%03d" % j, Params(k=51), g, off, 150, n, 0.005, False, seed,
                        {"G": 3 * g0, "coverage": 30, "arrival_s": float(arrivals[j])})

    return arrivals, [lambda j=j: make(j) for j in range(n_jobs)]


WORKLOADS = {0: tiny, 1: mid, 2: human_share}
