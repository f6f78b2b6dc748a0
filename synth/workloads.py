"""The five synthetic workloads: genome recipe, read recipe and alignment parameters.

Stand-ins for the paper's inputs (Section 2: reads simulated from the human
reference with substitutions and indels; Table 1 = 100/200 bp, Table 2 = 1 kb /
10 kb with 20% indels). The paper's data (hg19, simulated read sets, NA12878)
is not available, so every genome and read set here is seeded and synthetic.

The parameter values (s, n, d_max, c, h_max) are not given by the paper for any
experiment (Table 3 only names them); the values below are readings: s = 20 and
c = 2 throughout, n(L) = min(32, max(10, ceil(L / 100))), h_max = 300, and d_max 8
(tiny), 10 (mid), 15 (human scale) or max(8, ceil(8 L / 100)) (mixed long reads).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from . import ReadModel, Reads, genome_repeats, genome_uniform, simulate_reads


@dataclass(frozen=True)
class Params:
    """Alignment parameters (Table 3) plus the read-length rules for n and d_max."""
    seed_len: int = 20         # s
    n_min: int = 10            # n(L) = min(n_cap, max(n_min, ceil(L / bp_per_seed)))
    n_cap: int = 32
    bp_per_seed: int = 100
    conf_c: int = 2            # c
    max_hits: int = 300        # h_max
    d_max: int = 8             # d_max(L) = max(d_max, ceil(d_max_pct * L / 100))
    d_max_pct: int = 0
    bucket: int = 32           # merge bucket (omitted aspect 1 of Section 3.2)


@dataclass
class Workload:
    name: str
    genome_len: int
    genome_seed: int
    genome_kind: str           # "uniform" | "repeats"
    n_frac: float
    n_reads: int
    read_seed: int
    reads: ReadModel
    params: Params
    notes: str = ""

    def make_genome(self) -> np.ndarray:
        if self.genome_kind == "uniform":
            return genome_uniform(self.genome_len, self.genome_seed)
        return genome_repeats(self.genome_len, self.genome_seed, n_frac=self.n_frac)

    def make_reads(self, genome: np.ndarray, n: int | None = None) -> Reads:
        return simulate_reads(genome, self.n_reads if n is None else n, self.read_seed, self.reads)

    def scaled(self, genome_len: int | None = None, n_reads: int | None = None) -> "Workload":
        """Same recipe at another size (for tests the oracle finishes in seconds)."""
        return replace(self, genome_len=genome_len or self.genome_len, n_reads=n_reads or self.n_reads)


TINY = Workload(
    name="tiny", genome_len=1_000_000, genome_seed=0, genome_kind="uniform", n_frac=0.0,
    n_reads=10_000, read_seed=100,
    reads=ReadModel(len_mode=0, len_a=100, len_b=100, p_sub=0.005, p_indel=0.0005, indel_max=5),
    params=Params(d_max=8),
    notes="1 Mbase uniform genome, 10k x 100 bp, 0.5% subs, 0.05% indels (1-5)")

MID = Workload(
    name="mid", genome_len=100_000_000, genome_seed=1, genome_kind="repeats", n_frac=0.0,
    n_reads=10_000_000, read_seed=101,
    reads=ReadModel(len_mode=0, len_a=100, len_b=100, p_sub=0.01, p_indel=0.001, indel_max=5),
    params=Params(d_max=10),
    notes="100 Mbase, 50% repeats (40% segdup, 10% tandem), 10M x 100 bp, 1% subs, 0.1% indels")

HUMAN = Workload(
    name="human", genome_len=3_100_000_000, genome_seed=2, genome_kind="repeats", n_frac=0.01,
    n_reads=100_000_000, read_seed=102,
    reads=ReadModel(len_mode=1, len_a=100, len_b=250, p_sub=0.01, p_indel=0.002, indel_max=10),
    params=Params(d_max=15),
    notes="3.1 Gbase, repeats + 1% N-runs, 100M reads of 100/250 bp, 1% subs, 0.2% indels (1-10)")

BATCHED = Workload(
    name="batched", genome_len=3_100_000_000, genome_seed=2, genome_kind="repeats", n_frac=0.01,
    n_reads=5_000_000, read_seed=103,
    reads=ReadModel(len_mode=2, len_a=100, len_b=10_000, p_sub=0.008, p_indel=0.002, indel_max=10,
                    p_sub_long=0.025, p_indel_long=0.025, indel_max_long=5, long_thr=300),
    params=Params(d_max=8, d_max_pct=8),
    notes="5M reads, log-uniform 100 bp-10 kb; <=300 bp 1% error, longer 5% (half indels); d_max=ceil(0.08 L)")

SERVED = Workload(
    name="served", genome_len=3_100_000_000, genome_seed=2, genome_kind="repeats", n_frac=0.01,
    n_reads=1_000_000, read_seed=104,
    reads=BATCHED.reads,
    params=BATCHED.params,
    notes="requests of floor(10^(4u)) reads drawn from a pool with the batched length/error mix; Poisson arrivals")

WORKLOADS = {w.name: w for w in (TINY, MID, HUMAN, BATCHED, SERVED)}
