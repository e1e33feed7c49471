"""Seeded LDA corpora in CSR form.

The generative process is the one the paper uses for its simulations
(Appendix, "Simulation Data Generation Process"): every topic is a word
distribution mu_k ~ Dirichlet over the vocabulary, every document draws a topic
mixture h_d ~ Dirichlet(alpha), and each of its L_d tokens draws a topic
z ~ Cat(h_d) and then a word w ~ Cat(mu_z).

Tweet-shaped workloads add two things the paper's corpora have and its
simulation does not spell out: a Zipf background mixed into every topic
(word ids come from a seeded permutation of the Zipf ranks, so frequent words
are not ids 0..k), and document lengths L_d = 1 + Poisson(lambda).

Determinism: topics come from one child of SeedSequence(seed); documents are
generated in chunks of 65 536, chunk c from child c + 1, so the corpus is the
same at any thread count and any batch size.

Small Dirichlet concentrations (0.01 over 20 000 words) underflow a plain Gamma
sampler, so Gamma(a) draws are taken in log space:
log G(a) = log G(a + 1) + log(U) / a   (Marsaglia & Tsang's boost identity).
"""
from __future__ import annotations

import dataclasses
from typing import Iterator, Optional

import numpy as np

CHUNK = 65536


@dataclasses.dataclass(frozen=True)
class CorpusSpec:
    name: str
    V: int
    K: int
    N: int
    doc_len_lambda: float          # L_d = 1 + Poisson(lambda)
    alpha0: float                  # Dirichlet(alpha0 / K * 1_K) document mixtures
    topic_conc: float              # Dirichlet(topic_conc * 1_V) topic components
    zipf_s: Optional[float]        # Zipf exponent of the background, None = no background
    zipf_mix: float                # weight of the background in every topic
    batch: int                     # documents per CSR batch
    seed: int

    @property
    def alpha(self) -> np.ndarray:
        return np.full(self.K, self.alpha0 / self.K)


SPECS = {
    # Plain TLDA, 500 words, 5 topics from Dirichlet(0.1), alpha = 0.2 per topic.
    "c1": CorpusSpec("c1", V=500, K=5, N=5000, doc_len_lambda=50.0, alpha0=1.0,
                     topic_conc=0.1, zipf_s=None, zipf_mix=0.0, batch=1000, seed=1001),
    # Tweet-shaped corpus: V = 20 000, 50 topics, 1M documents of ~21 tokens.
    "c2": CorpusSpec("c2", V=20000, K=50, N=1_000_000, doc_len_lambda=20.0, alpha0=1.0,
                     topic_conc=0.01, zipf_s=1.1, zipf_mix=0.3, batch=131072, seed=1002),
    # Streaming scale: V = 50 000, 100 topics, 20M documents of ~16 tokens.
    "c3": CorpusSpec("c3", V=50000, K=100, N=20_000_000, doc_len_lambda=15.0, alpha0=2.0,
                     topic_conc=0.01, zipf_s=1.05, zipf_mix=0.3, batch=262144, seed=1003),
}


def slice_specs(n_slices: int = 64, seed: int = 1004, median: float = 150_000.0,
                sigma: float = 1.0, lo: int = 10_000, hi: int = 2_000_000,
                scale: float = 1.0) -> list:
    """The batched-time-slice workload: independent corpora sharing V = 20 000,
    sizes clip(round(exp(N(ln median, sigma))), lo, hi) (times `scale`, for
    smaller runs), K drawn uniformly from {10, 20, 50}, tweet-shaped documents
    and topics as in c2, each slice with its own seed and planted topics."""
    rng = np.random.default_rng(seed)
    sizes = np.clip(np.round(np.exp(rng.normal(np.log(median), sigma, n_slices))), lo, hi)
    ks = rng.choice([10, 20, 50], size=n_slices)
    return [CorpusSpec(f"c4.{i}", V=20000, K=int(ks[i]), N=max(1, int(sizes[i] * scale)),
                       doc_len_lambda=20.0, alpha0=1.0, topic_conc=0.01, zipf_s=1.1,
                       zipf_mix=0.3, batch=131072, seed=seed * 1000 + i)
            for i in range(n_slices)]


@dataclasses.dataclass
class Corpus:
    spec: CorpusSpec
    indptr: np.ndarray     # int64 [N + 1]
    indices: np.ndarray    # int32 [nnz], strictly increasing within a row
    data: np.ndarray       # float32 [nnz], positive integer counts
    mu: np.ndarray         # float64 [V, K] planted topic-word matrix (columns sum to 1)
    alpha: np.ndarray      # float64 [K] Dirichlet parameter of the document mixtures

    @property
    def n_docs(self) -> int:
        return self.indptr.shape[0] - 1

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])


def _log_dirichlet(rng: np.random.Generator, conc: np.ndarray, rows: int) -> np.ndarray:
    """Rows of Dirichlet(conc) draws, computed through log-Gamma variates."""
    conc = np.asarray(conc, dtype=np.float64)
    g = rng.standard_gamma(conc + 1.0, size=(rows, conc.shape[0]))
    u = rng.random((rows, conc.shape[0]))
    logx = np.log(g) + np.log(u) / conc
    logx -= logx.max(axis=1, keepdims=True)
    x = np.exp(logx)
    x /= x.sum(axis=1, keepdims=True)
    return x


def planted_topics(spec: CorpusSpec, rng: np.random.Generator) -> np.ndarray:
    """V x K topic-word matrix of the workload (columns sum to one)."""
    comp = _log_dirichlet(rng, np.full(spec.V, spec.topic_conc), spec.K).T
    if spec.zipf_s is None or spec.zipf_mix == 0.0:
        return comp
    ranks = np.arange(1, spec.V + 1, dtype=np.float64)
    z = ranks ** (-spec.zipf_s)
    z /= z.sum()
    perm = rng.permutation(spec.V)
    zipf = np.empty(spec.V)
    zipf[perm] = z
    mu = spec.zipf_mix * zipf[:, None] + (1.0 - spec.zipf_mix) * comp
    return mu / mu.sum(axis=0, keepdims=True)


def _chunk_docs(spec: CorpusSpec, cum_mu: np.ndarray, alpha: np.ndarray,
                rng: np.random.Generator, n: int):
    L = 1 + rng.poisson(spec.doc_len_lambda, size=n)
    h = _log_dirichlet(rng, alpha, n)
    cum_h = np.cumsum(h, axis=1)
    doc = np.repeat(np.arange(n, dtype=np.int64), L)
    u = rng.random(doc.shape[0])
    # topic of each token: inverse CDF of its document's mixture
    topic = np.empty(doc.shape[0], dtype=np.int64)
    step = 1 << 20
    for s in range(0, doc.shape[0], step):
        e = min(s + step, doc.shape[0])
        topic[s:e] = (cum_h[doc[s:e]] < u[s:e, None]).sum(axis=1)
    np.minimum(topic, spec.K - 1, out=topic)
    u2 = rng.random(doc.shape[0])
    word = np.empty(doc.shape[0], dtype=np.int64)
    order = np.argsort(topic, kind="stable")
    bounds = np.searchsorted(topic[order], np.arange(spec.K + 1))
    for k in range(spec.K):
        sel = order[bounds[k]:bounds[k + 1]]
        if sel.size:
            word[sel] = np.searchsorted(cum_mu[k], u2[sel], side="right")
    np.minimum(word, spec.V - 1, out=word)
    key = doc * spec.V + word
    uniq, counts = np.unique(key, return_counts=True)
    rows = uniq // spec.V
    cols = (uniq % spec.V).astype(np.int32)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    np.cumsum(indptr, out=indptr)
    return indptr, cols, counts.astype(np.float32)


_POOL_STATE = {}


def _pool_chunk(job):
    spec, cum_mu, alpha = _POOL_STATE["args"]
    child, n = job
    return _chunk_docs(spec, cum_mu, alpha, np.random.default_rng(child), n)


def generate(spec: CorpusSpec, n_docs: Optional[int] = None, workers: int = 1) -> Corpus:
    """Generate the first ``n_docs`` documents (default: all) of the workload.
    Chunks are independent (each has its own child seed), so ``workers`` > 1
    generates them in forked processes; the corpus is the same either way."""
    n_docs = spec.N if n_docs is None else int(n_docs)
    n_chunks = max(1, -(-n_docs // CHUNK))
    ss = np.random.SeedSequence(spec.seed)
    children = ss.spawn(n_chunks + 1)
    topic_rng = np.random.default_rng(children[0])
    mu = planted_topics(spec, topic_rng)
    cum_mu = np.cumsum(mu.T, axis=1)
    cum_mu[:, -1] = 1.0
    alpha = spec.alpha
    jobs = [(children[c + 1], min(CHUNK, n_docs - c * CHUNK)) for c in range(n_chunks)]
    if workers > 1 and n_chunks > 1:
        import multiprocessing as mp
        _POOL_STATE["args"] = (spec, cum_mu, alpha)
        pool = mp.get_context("fork").Pool(min(workers, n_chunks))
        try:
            chunks = pool.map(_pool_chunk, jobs)
            pool.close()   # the workers leave on their own, without a signal
        except BaseException:
            pool.terminate()
            raise
        finally:
            pool.join()
            _POOL_STATE.clear()
    else:
        chunks = [_chunk_docs(spec, cum_mu, alpha, np.random.default_rng(ch), n) for ch, n in jobs]
    ptrs, cols, vals = [], [], []
    offset = 0
    for ip, ci, va in chunks:
        ptrs.append(ip[1:] + offset)
        cols.append(ci)
        vals.append(va)
        offset += int(ip[-1])
    indptr = np.concatenate([np.zeros(1, dtype=np.int64)] + ptrs)
    return Corpus(spec, indptr, np.concatenate(cols), np.concatenate(vals), mu, alpha)


def make_csr_rows(rows, V: int):
    """CSR arrays (int32 row_ptr, int32 col_idx, float32 val) from a list of
    {word: count} dicts; used to build hand-made edge cases."""
    row_ptr = [0]
    col, val = [], []
    for r in rows:
        for w in sorted(r):
            if not (0 <= w < V):
                raise ValueError("word id out of range")
            col.append(w)
            val.append(float(r[w]))
        row_ptr.append(len(col))
    return (np.asarray(row_ptr, dtype=np.int32), np.asarray(col, dtype=np.int32),
            np.asarray(val, dtype=np.float32))


def iter_batches(corpus: Corpus, batch: Optional[int] = None) -> Iterator[tuple]:
    """Yield (row_ptr int32 rebased to 0, col_idx int32, val float32, first_doc)."""
    batch = corpus.spec.batch if batch is None else int(batch)
    N = corpus.n_docs
    for s in range(0, N, batch):
        e = min(s + batch, N)
        a, b = int(corpus.indptr[s]), int(corpus.indptr[e])
        rp = (corpus.indptr[s:e + 1] - a).astype(np.int32)
        yield rp, corpus.indices[a:b], corpus.data[a:b], s


def init_phi(D: int, K: int, seed: int) -> np.ndarray:
    """Initial CP factors, D x K.  The paper leaves the start point open; this
    draws a seeded Gaussian matrix and orthonormalises its columns (K <= D) or
    normalises them (K > D)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, D, K]))
    g = rng.standard_normal((D, K))
    if K <= D:
        q, r = np.linalg.qr(g)
        q *= np.sign(np.diag(r))[None, :]
        return q
    return g / np.linalg.norm(g, axis=0, keepdims=True)
