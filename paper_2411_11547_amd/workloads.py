"""Seeded synthetic read/haplotype batches shaped like the paper's workloads.

The paper measures on synthetic equal-length batches and on two real datasets
(GATK HaplotypeCaller batches from NA12878, and the small "10s" set; Section
IV-A).  Neither dataset is available, so every input here is generated from a
fixed seed with the shapes of those workloads: regions of candidate haplotypes
that are mutated copies of a reference, reads drawn from the haplotypes with
sequencing errors, and per-base Phred qualities.

This module holds none of the Pair-HMM arithmetic.  It produces bases as codes
(A=0, C=1, G=2, T=3, N=4) and qualities as Phred bytes only; turning those into
probabilities is the job of the oracle on one side and of the HIP kernels on
the other.  Both sides consume the same `Problem`.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

A, C, G, T, N = 0, 1, 2, 3, 4
CODE_OF = {"A": A, "C": C, "G": G, "T": T, "N": N}
CHAR_OF = "ACGTN"


@dataclass
class Problem:
    """A list of batches B_q = (R_q, H_q), every read of a batch against every
    haplotype of the same batch (Section II-A).  CSR layout:

    * reads of batch q are ``batch_read_begin[q] .. batch_read_begin[q+1]-1``;
    * haplotypes of batch q are ``batch_hap_begin[q] .. batch_hap_begin[q+1]-1``;
    * read r occupies ``read_offset[r] .. read_offset[r+1]-1`` of the per-base
      arrays (bases, base/ins/del/gap-continuation Phred);
    * haplotype h occupies ``hap_offset[h] .. hap_offset[h+1]-1`` of hap_bases.

    Output order: pair (q, r, h) with r, h local to the batch lands at
    ``out_offset[q] + r*|H_q| + h``, ``out_offset`` the exclusive scan of
    ``|R_q|*|H_q|``.
    """

    batch_read_begin: np.ndarray
    batch_hap_begin: np.ndarray
    read_offset: np.ndarray
    read_bases: np.ndarray
    base_qual: np.ndarray
    ins_qual: np.ndarray
    del_qual: np.ndarray
    gcp_qual: np.ndarray
    hap_offset: np.ndarray
    hap_bases: np.ndarray
    name: str = "custom"
    recipe: dict = field(default_factory=dict)

    def __post_init__(self):
        self.batch_read_begin = np.ascontiguousarray(self.batch_read_begin, dtype=np.int32)
        self.batch_hap_begin = np.ascontiguousarray(self.batch_hap_begin, dtype=np.int32)
        self.read_offset = np.ascontiguousarray(self.read_offset, dtype=np.int64)
        self.hap_offset = np.ascontiguousarray(self.hap_offset, dtype=np.int64)
        for f in ("read_bases", "base_qual", "ins_qual", "del_qual", "gcp_qual", "hap_bases"):
            setattr(self, f, np.ascontiguousarray(getattr(self, f), dtype=np.uint8))
        self._pairs = None

    # --- shape --------------------------------------------------------------
    @property
    def num_batches(self) -> int:
        return len(self.batch_read_begin) - 1

    @property
    def num_reads(self) -> int:
        return len(self.read_offset) - 1

    @property
    def num_haps(self) -> int:
        return len(self.hap_offset) - 1

    @property
    def read_lengths(self) -> np.ndarray:
        return np.diff(self.read_offset)

    @property
    def hap_lengths(self) -> np.ndarray:
        return np.diff(self.hap_offset)

    def batch_pair_counts(self) -> np.ndarray:
        return (np.diff(self.batch_read_begin).astype(np.int64)
                * np.diff(self.batch_hap_begin).astype(np.int64))

    @property
    def num_pairs(self) -> int:
        return int(self.batch_pair_counts().sum())

    def pair_index(self):
        """(read index, haplotype index) of every pair, in output order."""
        if self._pairs is None:
            nr = np.diff(self.batch_read_begin).astype(np.int64)
            nh = np.diff(self.batch_hap_begin).astype(np.int64)
            cnt = nr * nh
            P = int(cnt.sum())
            q = np.repeat(np.arange(self.num_batches, dtype=np.int64), cnt)
            start = np.concatenate([[0], np.cumsum(cnt)[:-1]]).astype(np.int64)
            local = np.arange(P, dtype=np.int64) - start[q]
            r = self.batch_read_begin[q] + local // nh[q]
            h = self.batch_hap_begin[q] + local % nh[q]
            self._pairs = (r.astype(np.int32), h.astype(np.int32))
        return self._pairs

    def pair_cells(self) -> np.ndarray:
        r, h = self.pair_index()
        return self.read_lengths[r].astype(np.int64) * self.hap_lengths[h].astype(np.int64)

    @property
    def total_cells(self) -> int:
        nr_len = np.add.reduceat(self.read_lengths, self.batch_read_begin[:-1]) \
            if self.num_reads else np.zeros(0, np.int64)
        nh_len = np.add.reduceat(self.hap_lengths, self.batch_hap_begin[:-1]) \
            if self.num_haps else np.zeros(0, np.int64)
        # reduceat misbehaves on empty batches; fall back to the pair sum then.
        if (np.diff(self.batch_read_begin) == 0).any() or (np.diff(self.batch_hap_begin) == 0).any():
            return int(self.pair_cells().sum())
        return int((nr_len.astype(np.int64) * nh_len.astype(np.int64)).sum())

    # --- accessors ------------------------------------------------------------
    def read(self, r: int):
        a, b = self.read_offset[r], self.read_offset[r + 1]
        return (self.read_bases[a:b], self.base_qual[a:b], self.ins_qual[a:b],
                self.del_qual[a:b], self.gcp_qual[a:b])

    def hap(self, h: int):
        return self.hap_bases[self.hap_offset[h]:self.hap_offset[h + 1]]

    def select_pairs(self, out_idx) -> "Problem":
        """A new problem with one batch (1 read x 1 haplotype) per selected
        pair, in the order given; used to check sampled outputs one by one."""
        r_all, h_all = self.pair_index()
        out_idx = np.asarray(out_idx, dtype=np.int64)
        rs, hs = r_all[out_idx], h_all[out_idx]
        rl, hl = self.read_lengths, self.hap_lengths
        r_off = np.concatenate([[0], np.cumsum(rl[rs])]).astype(np.int64)
        h_off = np.concatenate([[0], np.cumsum(hl[hs])]).astype(np.int64)
        ridx = _ranges(self.read_offset[rs], rl[rs])
        hidx = _ranges(self.hap_offset[hs], hl[hs])
        k = len(out_idx)
        return Problem(np.arange(k + 1), np.arange(k + 1), r_off,
                       self.read_bases[ridx], self.base_qual[ridx], self.ins_qual[ridx],
                       self.del_qual[ridx], self.gcp_qual[ridx], h_off, self.hap_bases[hidx],
                       name=f"{self.name}[sample {k}]", recipe=dict(self.recipe))


def _ranges(starts, lengths) -> np.ndarray:
    """Concatenated index ranges [s, s+l) for every (s, l)."""
    starts = np.asarray(starts, dtype=np.int64)
    lengths = np.asarray(lengths, dtype=np.int64)
    tot = int(lengths.sum())
    if tot == 0:
        return np.zeros(0, dtype=np.int64)
    rep = np.repeat(starts - np.concatenate([[0], np.cumsum(lengths)[:-1]]), lengths)
    return rep + np.arange(tot, dtype=np.int64)


# ---------------------------------------------------------------------------
# sampling helpers (bases and Phred bytes only)
# ---------------------------------------------------------------------------
def random_bases(rng, n: int) -> np.ndarray:
    return rng.integers(0, 4, size=n, dtype=np.uint8)


def substitute(rng, seq: np.ndarray, rate: float) -> np.ndarray:
    """Replace each base with probability ``rate`` by one of the 3 others."""
    out = seq.copy()
    hit = rng.random(len(seq)) < rate
    out[hit] = (out[hit] + rng.integers(1, 4, size=int(hit.sum()), dtype=np.uint8)) % 4
    return out


def mutate_haplotype(rng, ref: np.ndarray) -> np.ndarray:
    """Haplotype = reference with, at probability 1/2, 0-3 SNPs at distinct
    positions, otherwise one insertion or deletion of 1-5 bases at a uniform
    interior position."""
    n = len(ref)
    if rng.random() < 0.5:
        k = int(rng.integers(0, 4))
        out = ref.copy()
        if k:
            pos = rng.choice(n, size=k, replace=False)
            out[pos] = (out[pos] + rng.integers(1, 4, size=k, dtype=np.uint8)) % 4
        return out
    length = int(rng.integers(1, 6))
    if rng.random() < 0.5:  # insertion
        at = int(rng.integers(1, n))
        return np.concatenate([ref[:at], random_bases(rng, length), ref[at:]])
    at = int(rng.integers(1, n - length))
    return np.concatenate([ref[:at], ref[at + length:]])


def illumina_quals(rng, size) -> np.ndarray:
    """Illumina-like base qualities: 5% U{2..12}, 60% exactly 37 and 35%
    U{13..41} without 37, so the mode is 37 and 5% are at most Q12."""
    u = rng.random(size)
    low = rng.integers(2, 13, size=size)
    high = rng.integers(13, 41, size=size)  # 13..40, then skip 37
    high = np.where(high >= 37, high + 1, high)
    q = np.where(u < 0.05, low, np.where(u < 0.65, 37, high))
    return q.astype(np.uint8)


def _assemble(regions, name, recipe) -> Problem:
    """regions: list of (reads, haps); reads = list of (bases, bq, iq, dq, gq)."""
    rb, hb = [0], [0]
    rl, hl = [], []
    cols = [[] for _ in range(5)]
    haps = []
    for reads, hs in regions:
        for rd in reads:
            for c, a in zip(cols, rd):
                c.append(a)
            rl.append(len(rd[0]))
        for h in hs:
            haps.append(h)
            hl.append(len(h))
        rb.append(rb[-1] + len(reads))
        hb.append(hb[-1] + len(hs))
    cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0, np.uint8)
    return Problem(np.array(rb), np.array(hb),
                   np.concatenate([[0], np.cumsum(rl)]).astype(np.int64),
                   cat(cols[0]), cat(cols[1]), cat(cols[2]), cat(cols[3]), cat(cols[4]),
                   np.concatenate([[0], np.cumsum(hl)]).astype(np.int64), cat(haps),
                   name=name, recipe=recipe)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------
def config0(seed: int = 0) -> Problem:
    """1 region: 150 bp reference, 4 mutated haplotypes (145-155 bp), 8 reads
    of 100 bp with 1% substitutions; base Q U{10..40}, ins = del = 45, gcp 10."""
    rng = np.random.default_rng(seed)
    ref = random_bases(rng, 150)
    haps = [mutate_haplotype(rng, ref) for _ in range(4)]
    reads = []
    for _ in range(8):
        h = haps[int(rng.integers(0, 4))]
        s = int(rng.integers(0, len(h) - 100 + 1))
        b = substitute(rng, h[s:s + 100], 0.01)
        reads.append((b, rng.integers(10, 41, size=100).astype(np.uint8),
                      np.full(100, 45, np.uint8), np.full(100, 45, np.uint8),
                      np.full(100, 10, np.uint8)))
    return _assemble([(reads, haps)], "plain-fp32-32pairs",
                     {"regions": 1, "reads": 8, "haps": 4, "read_len": 100,
                      "hap_len": "145-155", "base_q": "U{10..40}", "ins_del_q": 45, "gcp": 10})


def _region(rng, ref_len, trunc, n_haps, read_lens):
    ref = random_bases(rng, ref_len)
    haps = []
    for _ in range(n_haps):
        h = mutate_haplotype(rng, ref)
        haps.append(h[:trunc] if trunc is not None else h)
    R = len(read_lens)
    choice = rng.integers(0, n_haps, size=R)
    reads = []
    bq_all = illumina_quals(rng, int(np.sum(read_lens)))
    iq_all = rng.integers(40, 46, size=int(np.sum(read_lens))).astype(np.uint8)
    dq_all = rng.integers(40, 46, size=int(np.sum(read_lens))).astype(np.uint8)
    o = 0
    for i in range(R):
        h = haps[choice[i]]
        L = int(min(read_lens[i], len(h)))
        s = int(rng.integers(0, len(h) - L + 1))
        b = substitute(rng, h[s:s + L], 0.01)
        reads.append((b, bq_all[o:o + L], iq_all[o:o + L], dq_all[o:o + L],
                      np.full(L, 10, np.uint8)))
        o += L
    return reads, haps


def config1(seed: int = 1, regions: int = 1000) -> Problem:
    """Uniform batch: regions x (64 reads of 150 bp x 8 haplotypes of 300 bp);
    Illumina-like base Q, ins/del Phred U{40..45}, gcp 10."""
    rng = np.random.default_rng(seed)
    regs = [_region(rng, 310, 300, 8, np.full(64, 150)) for _ in range(regions)]
    return _assemble(regs, f"uniform-{regions}x64x8-150x300",
                     {"regions": regions, "reads": 64, "haps": 8, "read_len": 150,
                      "hap_len": 300, "base_q": "illumina-like", "ins_del_q": "U{40..45}",
                      "gcp": 10})


def config2(seed: int = 2, regions: int = 2000) -> Problem:
    """Mixed lengths: per region H = min(Geom(1/8), 64) haplotypes of length
    clip(round(LogNormal(ln 350, 0.5)), 100, 2000), R = round(10^U(1,3))
    reads of length U{50..250} (clipped to the haplotype)."""
    rng = np.random.default_rng(seed)
    regs = []
    for _ in range(regions):
        H = int(min(rng.geometric(1 / 8), 64))
        R = int(round(10 ** rng.uniform(1, 3)))
        n_r = int(np.clip(round(rng.lognormal(np.log(350), 0.5)), 100, 2000))
        lens = rng.integers(50, 251, size=R)
        regs.append(_region(rng, n_r + 10, n_r, H, lens))
    return _assemble(regs, f"mixed-{regions}regions",
                     {"regions": regions, "haps": "min(Geom(1/8),64)", "reads": "round(10^U(1,3))",
                      "read_len": "U{50..250}", "hap_len": "clip(LogNormal(ln350,0.5),100,2000)",
                      "base_q": "illumina-like", "ins_del_q": "U{40..45}", "gcp": 10})


def config3(seed: int = 3, pairs: int = 50000) -> Problem:
    """Precision stress: independent pairs, haplotype n ~ U{1000..5000} at SNP
    divergence U(0.05, 0.15) from a reference; read = 250 bp of the reference
    with 1% errors and 2% N; 30% of reads have all base Q in U{2..10}."""
    rng = np.random.default_rng(seed)
    n = rng.integers(1000, 5001, size=pairs).astype(np.int64)
    ref = random_bases(rng, int(n.sum()))
    div = np.repeat(rng.uniform(0.05, 0.15, size=pairs), n)
    hit = rng.random(len(ref)) < div
    hap = ref.copy()
    hap[hit] = (hap[hit] + rng.integers(1, 4, size=int(hit.sum()), dtype=np.uint8)) % 4
    h_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    m = 250
    start = h_off[:-1] + (rng.random(pairs) * (n - m + 1)).astype(np.int64)
    rd = ref[_ranges(start, np.full(pairs, m))]
    rd = substitute(rng, rd, 0.01)
    rd[rng.random(len(rd)) < 0.02] = N
    low = np.repeat(rng.random(pairs) < 0.30, m)
    bq = np.where(low, rng.integers(2, 11, size=len(rd)), illumina_quals(rng, len(rd))).astype(np.uint8)
    iq = rng.integers(40, 46, size=len(rd)).astype(np.uint8)
    dq = rng.integers(40, 46, size=len(rd)).astype(np.uint8)
    gq = np.full(len(rd), 10, np.uint8)
    idx = np.arange(pairs + 1)
    return Problem(idx, idx, np.arange(pairs + 1, dtype=np.int64) * m, rd, bq, iq, dq, gq,
                   h_off, hap, name=f"precision-stress-{pairs}pairs-250x1000..5000",
                   recipe={"pairs": pairs, "read_len": 250, "hap_len": "U{1000..5000}",
                           "divergence": "U(0.05,0.15)", "N_rate": 0.02,
                           "low_q_reads": "30% U{2..10}"})


def config4(seed: int = 4, pairs: int = 10000) -> Problem:
    """Adjoint workload: independent pairs, haplotype = mutated reference of
    length U{200..600} (so 195..605 bases after an indel); read = 150 bp of
    the unmutated reference with 1% errors; Illumina-like base Q, ins/del
    U{40..45}, gcp 10."""
    rng = np.random.default_rng(seed)
    regs = []
    for _ in range(pairs):
        n = int(rng.integers(200, 601))
        ref = random_bases(rng, n)
        h = mutate_haplotype(rng, ref)
        s = int(rng.integers(0, n - 150 + 1))
        b = substitute(rng, ref[s:s + 150], 0.01)
        regs.append(([(b, illumina_quals(rng, 150),
                       rng.integers(40, 46, size=150).astype(np.uint8),
                       rng.integers(40, 46, size=150).astype(np.uint8),
                       np.full(150, 10, np.uint8))], [h]))
    return _assemble(regs, f"adjoint-{pairs}pairs-150x200..600",
                     {"pairs": pairs, "read_len": 150, "hap_len": "U{200..600}",
                      "base_q": "illumina-like", "ins_del_q": "U{40..45}", "gcp": 10})


def make(config: int, **kw) -> Problem:
    return [config0, config1, config2, config3, config4][config](**kw)


def from_strings(batches, base_q=20, ins_q=45, del_q=45, gcp_q=10) -> Problem:
    """Small problems from text: batches = [([read strings], [hap strings])].
    Qualities are constants (or per-read lists of per-base values)."""
    regions = []
    for reads, haps in batches:
        rr = []
        for s in reads:
            b = np.array([CODE_OF[ch] for ch in s], np.uint8)
            L = len(b)
            f = lambda q: np.asarray(q, np.uint8) if np.ndim(q) else np.full(L, q, np.uint8)
            rr.append((b, f(base_q), f(ins_q), f(del_q), f(gcp_q)))
        hh = [np.array([CODE_OF[ch] for ch in s], np.uint8) for s in haps]
        regions.append((rr, hh))
    return _assemble(regions, "from-strings", {})
