"""ctypes wrapper of the C oracle -- TEST INFRASTRUCTURE ONLY.

The oracle is the plain serial loop over individuals (Supplementary Fig.
S5(A)) of one replicate; batches of replicates are lists of ``OraclePop``.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SPEGG_ORACLE_LIB") or os.path.join(HERE, "libspegg_oracle.so")

ALWAYS = 1 << 32
MODE_NAMES = {0: "raw", 1: "zero", 2: "skip", 3: "lazy"}


class OracleEcology(C.Structure):
    _fields_ = [
        ("n0_consumer", C.c_uint32),
        ("capacity_consumer", C.c_uint32),
        ("resource_trials", C.c_uint32),
        ("habitat", C.c_uint32),
        ("attack", C.c_double),
        ("match_width", C.c_double),
        ("encounters", C.c_double),
        ("conversion", C.c_double),
        ("resource_q0", C.c_double),
        ("resource_K", C.c_double),
        ("surv_resource", C.c_double * 4),
        ("surv_consumer", C.c_double * 4),
    ]


def make_ecology(eco):
    e = OracleEcology()
    for k, v in eco.items():
        if k in ("surv_resource", "surv_consumer"):
            arr = getattr(e, k)
            for a in range(4):
                arr[a] = float(v[a])
        else:
            setattr(e, k, v)
    return e


class OraclePhysiology(C.Structure):
    _fields_ = [
        ("alpha", C.c_double), ("gamma", C.c_double), ("delta", C.c_double),
        ("attack", C.c_double), ("handling", C.c_double),
        ("K", C.c_double * 2), ("growth", C.c_double * 2), ("growth_sd", C.c_double * 2), ("R0", C.c_double * 2),
        ("steepness", C.c_double), ("switch_frac", C.c_double), ("w_max", C.c_double),
        ("kappa", C.c_double), ("qJ", C.c_double), ("qA", C.c_double),
        ("beta1", C.c_double), ("beta2", C.c_double), ("beta_s", C.c_double),
        ("maturity", C.c_double),
        ("v_f", C.c_double), ("v_m", C.c_double),
        ("kappa1", C.c_double), ("kappa2", C.c_double), ("kappa3", C.c_double),
        ("breed_every", C.c_uint32),
    ]


def make_physiology(phy):
    f = OraclePhysiology()
    for k, v in phy.items():
        if k in ("K", "growth", "growth_sd", "R0"):
            arr = getattr(f, k)
            arr[0], arr[1] = float(v[0]), float(v[1])
        else:
            setattr(f, k, v)
    return f


class OracleParams(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64),
        ("replicate_id", C.c_uint32),
        ("regime", C.c_uint32),
        ("n0", C.c_uint32),
        ("capacity", C.c_uint32),
        ("n_loci", C.c_uint32),
        ("n_patches", C.c_uint32),
        ("mu", C.c_double),
        ("r", C.c_double),
        ("theta", C.c_double),
        ("omega", C.c_double),
        ("K", C.c_double),
        ("fecundity", C.c_double),
        ("migration", C.c_double),
        ("dispersal", C.c_uint32),
        ("home_return", C.c_double),
        ("effects", C.POINTER(C.c_int8)),
        ("ecology", C.POINTER(OracleEcology)),
        ("genetics", C.c_uint32),
        ("allele_mean", C.c_double),
        ("allele_sd", C.c_double),
        ("mut_sd_factor", C.c_double),
        ("noise_sd", C.c_double),
        ("exp_transform", C.c_uint32),
        ("linkage", C.POINTER(C.c_double)),
        ("sexes", C.c_uint32),
        ("mating", C.c_uint32),
        ("pref_optimum", C.c_double),
        ("pref_width", C.c_double),
        ("monogamy", C.c_uint32),
        ("physiology", C.POINTER(OraclePhysiology)),
    ]


class OracleStats(C.Structure):
    _fields_ = [
        ("generation", C.c_uint32),
        ("n", C.c_uint32),
        ("n_parents", C.c_uint32),
        ("n_survivors", C.c_uint32),
        ("extinct", C.c_uint32),
        ("captures", C.c_uint32),
        ("sum_z", C.c_int64),
        ("sum_z2", C.c_int64),
        ("near_ties", C.c_uint64),
        ("truncated", C.c_uint64),
        ("sum_threshold", C.c_uint64),
        ("updates", C.c_uint64),
        ("sum_zf", C.c_double),
        ("sum_zf2", C.c_double),
        ("resource", C.c_double * 2),
        ("eggs", C.c_double),
    ]

    def as_dict(self):
        out = {name: getattr(self, name) for name, _ in self._fields_}
        out["resource"] = (self.resource[0], self.resource[1])
        return out


_lib = None


def load():
    """Load (building first if needed) the oracle library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from .build import build
        build()
    lib = C.CDLL(LIB_PATH)
    u32, u64, i32, vp = C.c_uint32, C.c_uint64, C.c_int32, C.c_void_p
    P64 = C.POINTER(C.c_uint64)
    P32 = C.POINTER(C.c_uint32)
    lib.oracle_philox4x32_10.argtypes = [P32, P32, P32]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_prob_threshold.argtypes = [C.c_double]
    lib.oracle_prob_threshold.restype = u64
    lib.oracle_poisson_thresholds.argtypes = [C.c_double, P64, C.c_int]
    lib.oracle_poisson_thresholds.restype = C.c_int
    lib.oracle_binomial_thresholds.argtypes = [u32, C.c_double, P64, C.c_int]
    lib.oracle_binomial_thresholds.restype = C.c_int
    lib.oracle_geometric_thresholds.argtypes = [C.c_double, u32, P64]
    lib.oracle_geometric_thresholds.restype = None
    lib.oracle_small_binomial_thresholds.argtypes = [u32, C.c_double, P64]
    lib.oracle_small_binomial_thresholds.restype = C.c_int
    lib.oracle_recomb_mode.argtypes = [C.c_double]
    lib.oracle_recomb_mode.restype = C.c_int
    lib.oracle_create.argtypes = [C.POINTER(OracleParams)]
    lib.oracle_create.restype = vp
    lib.oracle_destroy.argtypes = [vp]
    lib.oracle_destroy.restype = None
    lib.oracle_step.argtypes = [vp, u32]
    lib.oracle_step.restype = C.c_int
    lib.oracle_get_stats.argtypes = [vp, u32, C.POINTER(OracleStats)]
    lib.oracle_get_stats.restype = C.c_int
    lib.oracle_get_n.argtypes = [vp, u32]
    lib.oracle_get_n.restype = u32
    lib.oracle_get_generation.argtypes = [vp]
    lib.oracle_get_generation.restype = u32
    lib.oracle_get_demes.argtypes = [vp]
    lib.oracle_get_demes.restype = u32
    lib.oracle_get_newborns.argtypes = [vp, u32]
    lib.oracle_get_newborns.restype = u32
    lib.oracle_get_ages.argtypes = [vp, u32, C.POINTER(C.c_uint8), C.c_size_t]
    lib.oracle_get_ages.restype = C.c_int
    lib.oracle_get_intake.argtypes = [vp, P32, C.c_size_t]
    lib.oracle_get_intake.restype = C.c_int
    lib.oracle_get_mode.argtypes = [vp]
    lib.oracle_get_mode.restype = C.c_int
    lib.oracle_get_genomes.argtypes = [vp, u32, P32, C.c_size_t]
    lib.oracle_get_genomes.restype = C.c_int
    lib.oracle_set_genomes.argtypes = [vp, u32, P32, u32, u32]
    lib.oracle_set_genomes.restype = C.c_int
    lib.oracle_get_phenotypes.argtypes = [vp, u32, C.POINTER(i32), C.c_size_t]
    lib.oracle_get_phenotypes.restype = C.c_int
    lib.oracle_get_survivors.argtypes = [vp, u32, P32, C.c_size_t]
    lib.oracle_get_survivors.restype = u32
    lib.oracle_get_parents.argtypes = [vp, u32, P32, P32, P32, C.c_size_t]
    lib.oracle_get_parents.restype = C.c_int
    lib.oracle_sample_gametes.argtypes = [vp, C.POINTER(C.c_uint8), u32, u32, u32, C.c_int, C.POINTER(C.c_uint8)]
    lib.oracle_sample_gametes.restype = C.c_int
    lib.oracle_phenotype.argtypes = [vp, C.POINTER(C.c_uint8), C.POINTER(C.c_uint8)]
    lib.oracle_phenotype.restype = i32
    lib.oracle_skip_gap.argtypes = [C.c_double, u32, u32]
    lib.oracle_skip_gap.restype = u32
    lib.oracle_find_gap_word.argtypes = [u64, u32, C.c_double, u32, u32, u32, u32, u32, P32]
    lib.oracle_find_gap_word.restype = C.c_int
    PF = C.POINTER(C.c_float)
    lib.oracle_get_alleles.argtypes = [vp, u32, PF, C.c_size_t]
    lib.oracle_get_alleles.restype = C.c_int
    lib.oracle_set_alleles.argtypes = [vp, u32, PF, u32, u32]
    lib.oracle_set_alleles.restype = C.c_int
    lib.oracle_get_phenotypes_f.argtypes = [vp, u32, PF, C.c_size_t]
    lib.oracle_get_phenotypes_f.restype = C.c_int
    lib.oracle_sample_gametes_cont.argtypes = [vp, PF, u32, u32, u32, C.c_int, PF]
    lib.oracle_sample_gametes_cont.restype = C.c_int
    lib.oracle_phenotype_cont.argtypes = [vp, PF, PF, u32, u32, u32]
    lib.oracle_phenotype_cont.restype = C.c_float
    lib.oracle_normals.argtypes = [u64, u32, u32, u32, u32, u32, u32, C.POINTER(C.c_double)]
    lib.oracle_normals.restype = None
    lib.oracle_get_sexes.argtypes = [vp, u32, C.POINTER(C.c_uint8), C.c_size_t]
    lib.oracle_get_sexes.restype = C.c_int
    lib.oracle_get_body.argtypes = [vp, u32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_size_t]
    lib.oracle_get_body.restype = C.c_int
    _lib = lib
    return lib


def _p(arr, ctype):
    return arr.ctypes.data_as(C.POINTER(ctype))


def philox4x32_10(ctr, key):
    lib = load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def prob_threshold(p):
    return int(load().oracle_prob_threshold(float(p)))


def poisson_thresholds(lam, cap=1024):
    out = np.zeros(cap, dtype=np.uint64)
    n = load().oracle_poisson_thresholds(float(lam), _p(out, C.c_uint64), cap)
    return out[:n].copy()


def binomial_thresholds(L, mu, cap=1024):
    out = np.zeros(cap, dtype=np.uint64)
    n = load().oracle_binomial_thresholds(int(L), float(mu), _p(out, C.c_uint64), cap)
    return out[:n].copy()


def geometric_thresholds(r, n):
    out = np.zeros(max(int(n), 1), dtype=np.uint64)
    load().oracle_geometric_thresholds(float(r), int(n), _p(out, C.c_uint64))
    return out[: int(n)].copy()


def small_binomial_thresholds(n, q):
    out = np.zeros(int(n) + 1, dtype=np.uint64)
    k = load().oracle_small_binomial_thresholds(int(n), float(q), _p(out, C.c_uint64))
    return out[:k].copy()


def recomb_mode(r):
    return MODE_NAMES[load().oracle_recomb_mode(float(r))]


def skip_gap(r, L, x):
    """Geometric crossover gap of word x (smallest k with x < T_k, else L-1)."""
    return int(load().oracle_skip_gap(float(r), int(L), int(x)))


def normals(seed, c3, index, stream, gen, sub0, n):
    """Box-Muller deviates of Philox blocks (index, stream, gen, sub0 + k)."""
    out = np.zeros(int(n), dtype=np.float64)
    load().oracle_normals(int(seed), int(c3), int(index), int(stream), int(gen), int(sub0), int(n),
                          _p(out, C.c_double))
    return out


def find_gap_word(seed, c3, r, L, n_slots, t_begin, t_end, x_target):
    """First (t, j, stream, word, boundary) whose gamete walk consumes
    x_target with a crossover still to follow, or None.  Releases the GIL,
    so disjoint generation ranges can be searched from several threads."""
    out = np.zeros(5, dtype=np.uint32)
    found = load().oracle_find_gap_word(int(seed), int(c3), float(r), int(L), int(n_slots), int(t_begin),
                                        int(t_end), int(x_target), _p(out, C.c_uint32))
    return tuple(int(v) for v in out) if found else None


class OraclePop:
    """One replicate in the oracle: a ring of ``n_patches`` patches (one by
    default), or the two species of the consumer-resource regime
    (``ecology`` given; species 0 resource, 1 consumer).  Per-deme
    accessors take ``patch`` or ``species``; ``total_stats`` sums the census
    over the demes."""

    def __init__(self, seed=1, replicate_id=0, regime=0, n0=100, capacity=None, n_loci=64,
                 mu=0.0, r=0.5, theta=0.0, omega=0.0, K=0.0, fecundity=0.0, effects=None,
                 n_patches=1, migration=0.0, ecology=None, dispersal=0, home_return=0.0, genetics=0,
                 allele_mean=0.0, allele_sd=0.0, mut_sd_factor=0.0, noise_sd=0.0, exp_transform=0,
                 linkage=None, sexes=0, mating=0, pref_optimum=0.0, pref_width=0.0, monogamy=0, physiology=None):
        lib = load()
        self.L = int(n_loci)
        self.W = (self.L + 31) // 32
        self.n_patches = int(n_patches)
        self._effects = None
        eff_ptr = None
        if effects is not None:
            self._effects = np.ascontiguousarray(effects, dtype=np.int8)
            assert self._effects.shape == (self.L,)
            eff_ptr = _p(self._effects, C.c_int8)
        self._eco = make_ecology(ecology) if ecology is not None else None
        self._phy = make_physiology(physiology) if physiology is not None else None
        self._linkage = None
        link_ptr = None
        if linkage is not None:
            self._linkage = np.ascontiguousarray(linkage, dtype=np.float64)
            assert self._linkage.shape == (max(self.L - 1, 0),)
            link_ptr = _p(self._linkage, C.c_double)
        prm = OracleParams(seed=seed, replicate_id=replicate_id, regime=regime, n0=n0,
                           capacity=n0 if capacity is None else capacity, n_loci=n_loci, n_patches=n_patches,
                           mu=mu, r=r, theta=theta, omega=omega, K=K, fecundity=fecundity, migration=migration,
                           dispersal=dispersal, home_return=home_return, effects=eff_ptr,
                           ecology=C.pointer(self._eco) if self._eco is not None else None, genetics=genetics,
                           allele_mean=allele_mean, allele_sd=allele_sd, mut_sd_factor=mut_sd_factor,
                           noise_sd=noise_sd, exp_transform=exp_transform, linkage=link_ptr, sexes=sexes,
                           mating=mating, pref_optimum=pref_optimum, pref_width=pref_width, monogamy=monogamy,
                           physiology=C.pointer(self._phy) if self._phy is not None else None)
        self.continuous = int(genetics) == 1
        self.capacity = prm.capacity
        self._h = lib.oracle_create(C.byref(prm))
        if not self._h:
            raise ValueError("oracle_create rejected the parameters")
        self._lib = lib
        self.n_demes = int(lib.oracle_get_demes(self._h))

    def close(self):
        if self._h:
            self._lib.oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        self._lib.oracle_step(self._h, int(n))

    @staticmethod
    def _deme(patch, species):
        return int(patch) + int(species)  # one of them is 0: rings have one species, two species one patch

    @property
    def n(self):
        return int(self._lib.oracle_get_n(self._h, 0))

    def n_of(self, patch=0, species=0):
        return int(self._lib.oracle_get_n(self._h, self._deme(patch, species)))

    @property
    def generation(self):
        return int(self._lib.oracle_get_generation(self._h))

    @property
    def mode(self):
        return MODE_NAMES[self._lib.oracle_get_mode(self._h)]

    def stats(self, patch=0, species=0):
        s = OracleStats()
        assert self._lib.oracle_get_stats(self._h, self._deme(patch, species), C.byref(s)) == 0
        return s.as_dict()

    def total_stats(self):
        """The census summed over demes (generation: shared; extinct: all)."""
        per = [self.stats(k) for k in range(self.n_demes)]
        out = {k: sum(p[k] for p in per) for k in per[0] if k != "resource"}
        out["resource"] = per[0]["resource"]  # one patch carries resources (physiology regime)
        out["generation"] = per[0]["generation"]
        out["extinct"] = int(all(p["extinct"] for p in per))
        return out

    def genomes(self, patch=0, species=0):
        """Packed genomes, shape (n, 2, W) uint32."""
        d = self._deme(patch, species)
        n = self.n_of(d)
        out = np.zeros(max(n, 1) * 2 * self.W, dtype=np.uint32)
        assert self._lib.oracle_get_genomes(self._h, d, _p(out, C.c_uint32), out.size) == 0
        return out[: n * 2 * self.W].reshape(n, 2, self.W)

    def alleles(self, patch=0, species=0):
        """Unpacked alleles, shape (n, 2, L) uint8."""
        g = self.genomes(patch, species)
        bits = np.unpackbits(g.view(np.uint8).reshape(g.shape[0], 2, -1), axis=-1, bitorder="little")
        return bits[..., : self.L]

    def set_genomes(self, words, generation, patch=0, species=0):
        w = np.ascontiguousarray(words, dtype=np.uint32).reshape(-1)
        n = w.size // (2 * self.W)
        assert self._lib.oracle_set_genomes(self._h, self._deme(patch, species), _p(w, C.c_uint32), n,
                                            int(generation)) == 0

    def phenotypes(self, patch=0, species=0):
        d = self._deme(patch, species)
        n = self.n_of(d)
        out = np.zeros(max(n, 1), dtype=np.int32)
        assert self._lib.oracle_get_phenotypes(self._h, d, _p(out, C.c_int32), out.size) == 0
        return out[:n]

    def body(self, patch=0):
        """Physiology regime: (X, Y) float64 arrays, irreversible and reversible mass."""
        n = self.n_of(patch)
        X = np.zeros(max(n, 1), dtype=np.float64)
        Y = np.zeros(max(n, 1), dtype=np.float64)
        assert self._lib.oracle_get_body(self._h, int(patch), _p(X, C.c_double), _p(Y, C.c_double), X.size) == 0
        return X[:n], Y[:n]

    def sexes(self, patch=0, species=0):
        """Separate sexes: 0 female, 1 male, per individual."""
        d = self._deme(patch, species)
        n = self.n_of(d)
        out = np.zeros(max(n, 1), dtype=np.uint8)
        assert self._lib.oracle_get_sexes(self._h, d, _p(out, C.c_uint8), out.size) == 0
        return out[:n]

    def ages(self, patch=0, species=0):
        d = self._deme(patch, species)
        n = self.n_of(d)
        out = np.zeros(max(n, 1), dtype=np.uint8)
        assert self._lib.oracle_get_ages(self._h, d, _p(out, C.c_uint8), out.size) == 0
        return out[:n]

    def intake(self):
        """Consumers' credited captures in the last generation, by adult index."""
        n = self.stats(species=1)["n_parents"]
        out = np.zeros(max(n, 1), dtype=np.uint32)
        assert self._lib.oracle_get_intake(self._h, _p(out, C.c_uint32), out.size) == 0
        return out[:n]

    def survivors(self, patch=0, species=0):
        d = self._deme(patch, species)
        m = self._lib.oracle_get_survivors(self._h, d, None, 0)
        out = np.zeros(max(m, 1), dtype=np.uint32)
        self._lib.oracle_get_survivors(self._h, d, _p(out, C.c_uint32), out.size)
        return out[:m]

    def newborns(self, patch=0, species=0):
        return int(self._lib.oracle_get_newborns(self._h, self._deme(patch, species)))

    def parents(self, patch=0, with_source=False, species=0):
        """Mother and father of each newborn of the last generation (indices
        into the adults of its source patch) and, with_source, that patch."""
        d = self._deme(patch, species)
        n = self.newborns(d)
        mom = np.zeros(max(n, 1), dtype=np.uint32)
        dad = np.zeros(max(n, 1), dtype=np.uint32)
        src = np.zeros(max(n, 1), dtype=np.uint32)
        assert self._lib.oracle_get_parents(self._h, d, _p(mom, C.c_uint32), _p(dad, C.c_uint32),
                                            _p(src, C.c_uint32), mom.size) == 0
        if with_source:
            return mom[:n], dad[:n], src[:n]
        return mom[:n], dad[:n]

    def sample_gametes(self, parent_alleles, j0, count, gen=0, paternal=False):
        """Gametes (count, L) uint8 of a parent given as (2, L) alleles."""
        par = np.ascontiguousarray(parent_alleles, dtype=np.uint8).reshape(2 * self.L)
        out = np.zeros((count, self.L), dtype=np.uint8)
        self._lib.oracle_sample_gametes(self._h, _p(par, C.c_uint8), int(j0), int(count), int(gen),
                                        1 if paternal else 0, _p(out, C.c_uint8))
        return out

    def allele_values(self, patch=0, species=0):
        """Continuous alleles, shape (n, 2, L) float32."""
        d = self._deme(patch, species)
        n = self.n_of(d)
        out = np.zeros(max(n, 1) * 2 * self.L, dtype=np.float32)
        assert self._lib.oracle_get_alleles(self._h, d, _p(out, C.c_float), out.size) == 0
        return out[: n * 2 * self.L].reshape(n, 2, self.L)

    def set_allele_values(self, values, generation, patch=0, species=0):
        v = np.ascontiguousarray(values, dtype=np.float32).reshape(-1)
        n = v.size // (2 * self.L)
        assert self._lib.oracle_set_alleles(self._h, self._deme(patch, species), _p(v, C.c_float), n,
                                            int(generation)) == 0

    def phenotypes_f(self, patch=0, species=0):
        """Continuous alleles: expressed phenotypes, float32."""
        d = self._deme(patch, species)
        n = self.n_of(d)
        out = np.zeros(max(n, 1), dtype=np.float32)
        assert self._lib.oracle_get_phenotypes_f(self._h, d, _p(out, C.c_float), out.size) == 0
        return out[:n]

    def sample_gametes_cont(self, parent_values, j0, count, gen=0, paternal=False):
        """Continuous-allele gametes (count, L) float32 of a parent given as (2, L) values."""
        par = np.ascontiguousarray(parent_values, dtype=np.float32).reshape(2 * self.L)
        out = np.zeros((count, self.L), dtype=np.float32)
        assert self._lib.oracle_sample_gametes_cont(self._h, _p(par, C.c_float), int(j0), int(count), int(gen),
                                                    1 if paternal else 0, _p(out, C.c_float)) == 0
        return out

    def phenotype_cont_of(self, h0, h1, j=0, gen=0, sub=0):
        a = np.ascontiguousarray(h0, dtype=np.float32)
        b = np.ascontiguousarray(h1, dtype=np.float32)
        return float(self._lib.oracle_phenotype_cont(self._h, _p(a, C.c_float), _p(b, C.c_float), int(j), int(gen),
                                                     int(sub)))

    def phenotype_of(self, h0, h1):
        a = np.ascontiguousarray(h0, dtype=np.uint8)
        b = np.ascontiguousarray(h1, dtype=np.uint8)
        return int(self._lib.oracle_phenotype(self._h, _p(a, C.c_uint8), _p(b, C.c_uint8)))
