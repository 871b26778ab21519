"""Python binding of libspegg (include/spegg.h): argument marshalling only.

PyTorch supplies the device memory (one ``uint8`` tensor of
``spegg_footprint`` bytes) and the stream; every step of the generation runs
in the library's HIP kernels.  Loading fails loudly when the library is not
built: there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libspegg.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_STATE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
WF, POISSON_BH, CONSUMER_RESOURCE, PHYSIOLOGY = 0, 1, 2, 3
KERNEL_NAMES = ["survive", "compact", "offspring", "encounter", "carry"]


class SpeggError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"spegg status {status}: {message}")
        self.status = status


class Ecology(C.Structure):
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


class Physiology(C.Structure):
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
    f = Physiology()
    for k, v in phy.items():
        if k in ("K", "growth", "growth_sd", "R0"):
            arr = getattr(f, k)
            arr[0], arr[1] = float(v[0]), float(v[1])
        else:
            setattr(f, k, v)
    return f


class RepDesc(C.Structure):
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
        ("ecology", C.POINTER(Ecology)),
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
        ("physiology", C.POINTER(Physiology)),
    ]


class RepStats(C.Structure):
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
    """Load the built library; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(or python paper_1603_09255_amd/build.py) first")
    lib = C.CDLL(LIB_PATH)
    vp, u32, st = C.c_void_p, C.c_uint32, C.c_int
    P32 = C.POINTER(C.c_uint32)
    lib.spegg_abi_version.restype = C.c_int
    lib.spegg_abi_version.argtypes = []
    lib.spegg_last_error.restype = C.c_char_p
    lib.spegg_last_error.argtypes = []
    lib.spegg_footprint.restype = C.c_size_t
    lib.spegg_footprint.argtypes = [C.POINTER(RepDesc), u32]
    lib.spegg_pop_create.restype = st
    lib.spegg_pop_create.argtypes = [C.POINTER(RepDesc), u32, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.spegg_step_generations.restype = st
    lib.spegg_step_generations.argtypes = [vp, u32]
    lib.spegg_stats.restype = st
    lib.spegg_stats.argtypes = [vp, C.POINTER(RepStats), u32]
    lib.spegg_deme_stats.restype = st
    lib.spegg_deme_stats.argtypes = [vp, u32, C.POINTER(RepStats), u32]
    lib.spegg_read_genomes.restype = st
    lib.spegg_read_genomes.argtypes = [vp, u32, u32, u32, P32, C.c_size_t, P32]
    lib.spegg_write_genomes.restype = st
    lib.spegg_write_genomes.argtypes = [vp, u32, u32, u32, P32, u32, u32]
    lib.spegg_read_phenotypes.restype = st
    lib.spegg_read_phenotypes.argtypes = [vp, u32, u32, u32, C.POINTER(C.c_int32), C.c_size_t, P32]
    PF = C.POINTER(C.c_float)
    lib.spegg_read_alleles.restype = st
    lib.spegg_read_alleles.argtypes = [vp, u32, u32, PF, C.c_size_t, P32]
    lib.spegg_write_alleles.restype = st
    lib.spegg_write_alleles.argtypes = [vp, u32, u32, PF, u32, u32]
    lib.spegg_read_phenotypes_f.restype = st
    lib.spegg_read_phenotypes_f.argtypes = [vp, u32, u32, PF, C.c_size_t, P32]
    lib.spegg_read_body.restype = st
    lib.spegg_read_body.argtypes = [vp, u32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_size_t, P32]
    lib.spegg_read_sexes.restype = st
    lib.spegg_read_sexes.argtypes = [vp, u32, u32, C.POINTER(C.c_uint8), C.c_size_t, P32]
    lib.spegg_read_ages.restype = st
    lib.spegg_read_ages.argtypes = [vp, u32, u32, C.POINTER(C.c_uint8), C.c_size_t, P32]
    lib.spegg_read_intake.restype = st
    lib.spegg_read_intake.argtypes = [vp, u32, P32, C.c_size_t, P32]
    lib.spegg_read_survivors.restype = st
    lib.spegg_read_survivors.argtypes = [vp, u32, u32, u32, P32, C.c_size_t, P32]
    lib.spegg_allele_counts.restype = st
    lib.spegg_allele_counts.argtypes = [vp, u32, u32, u32, vp, P32, u32, P32]
    lib.spegg_allele_counts_noalloc.restype = st
    lib.spegg_allele_counts_noalloc.argtypes = [vp, u32, u32, u32, P32, u32, P32]
    lib.spegg_set_trace.restype = st
    lib.spegg_set_trace.argtypes = [vp, C.c_int]
    lib.spegg_read_parents.restype = st
    lib.spegg_read_parents.argtypes = [vp, u32, u32, u32, P32, P32, P32, C.c_size_t, P32]
    lib.spegg_autotune.restype = st
    lib.spegg_autotune.argtypes = [vp, u32, P32, P32, u32, P32]
    lib.spegg_set_offspring_cap.restype = st
    lib.spegg_set_offspring_cap.argtypes = [vp, u32, u32]
    lib.spegg_set_graph.restype = st
    lib.spegg_set_graph.argtypes = [vp, C.c_int]
    lib.spegg_set_timing.restype = st
    lib.spegg_set_timing.argtypes = [vp, u32]
    lib.spegg_offspring_class_times.restype = st
    lib.spegg_offspring_class_times.argtypes = [vp, P32, P32, C.POINTER(C.c_double), C.POINTER(C.c_uint64), u32, P32]
    lib.spegg_prepare_graphs.restype = st
    lib.spegg_prepare_graphs.argtypes = [vp]
    lib.spegg_kernel_times.restype = st
    lib.spegg_kernel_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_uint64), u32]
    lib.spegg_pop_destroy.restype = None
    lib.spegg_pop_destroy.argtypes = [vp]
    lib.spegg_threshold_table.restype = C.c_int
    lib.spegg_threshold_table.argtypes = [C.c_int, C.c_double, u32, C.POINTER(C.c_uint64), C.c_int]
    lib.spegg_recomb_mode.restype = C.c_int
    lib.spegg_recomb_mode.argtypes = [C.c_double]
    lib.spegg_geometric_gap.restype = C.c_int
    lib.spegg_geometric_gap.argtypes = [C.c_double, u32, u32, u32, P32]
    lib.spegg_philox_fill.restype = st
    lib.spegg_philox_fill.argtypes = [C.c_uint64, vp, vp, u32, vp]
    lib.spegg_philox_rate.restype = st
    lib.spegg_philox_rate.argtypes = [C.c_uint64, u32, vp, u32, vp]
    lib.spegg_server_create.restype = st
    lib.spegg_server_create.argtypes = [vp, C.c_size_t, vp, u32, C.POINTER(vp)]
    lib.spegg_server_submit.restype = st
    lib.spegg_server_submit.argtypes = [vp, C.c_uint64, C.POINTER(RepDesc), u32, u32]
    lib.spegg_server_step.restype = st
    lib.spegg_server_step.argtypes = [vp, u32, P32, P32]
    lib.spegg_server_poll.restype = st
    lib.spegg_server_poll.argtypes = [vp, C.POINTER(C.c_uint64), u32, P32]
    lib.spegg_server_result.restype = st
    lib.spegg_server_result.argtypes = [vp, C.c_uint64, C.POINTER(RepStats), u32]
    lib.spegg_server_usage.restype = st
    lib.spegg_server_usage.argtypes = [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    lib.spegg_server_keep.restype = st
    lib.spegg_server_keep.argtypes = [vp, C.c_uint64]
    lib.spegg_server_population.restype = st
    lib.spegg_server_population.argtypes = [vp, C.c_uint64, C.POINTER(vp)]
    lib.spegg_server_release.restype = st
    lib.spegg_server_release.argtypes = [vp, C.c_uint64]
    lib.spegg_server_destroy.restype = None
    lib.spegg_server_destroy.argtypes = [vp]
    _lib = lib
    return lib


def last_error():
    return load().spegg_last_error().decode()


def check(status):
    if status != OK:
        raise SpeggError(status, last_error())


def _p(arr, ctype):
    return arr.ctypes.data_as(C.POINTER(ctype))


DESC_KEYS = ("seed", "replicate_id", "regime", "n0", "capacity", "n_loci", "mu", "r", "theta", "omega", "K",
             "fecundity", "effects", "n_patches", "migration", "ecology", "dispersal", "home_return", "genetics",
             "allele_mean", "allele_sd", "mut_sd_factor", "noise_sd", "exp_transform", "linkage", "sexes", "mating",
             "pref_optimum", "pref_width", "monogamy", "physiology")
RING, ISLAND = 0, 1
BIALLELIC, CONTINUOUS = 0, 1
RANDOM_MATING, PREFERENCE, ASSORTATIVE = 0, 1, 2


def make_ecology(eco):
    e = Ecology()
    for k, v in eco.items():
        if k in ("surv_resource", "surv_consumer"):
            arr = getattr(e, k)
            for a in range(4):
                arr[a] = float(v[a])
        else:
            setattr(e, k, v)
    return e


def make_descs(reps):
    """ctypes array of descriptors from dicts; returns (array, keepalive)."""
    arr = (RepDesc * len(reps))()
    keep = []
    for k, d in enumerate(reps):
        unknown = set(d) - set(DESC_KEYS)
        if unknown:
            raise ValueError(f"unknown descriptor keys {sorted(unknown)}")
        n0 = int(d.get("n0", 0))
        arr[k].seed = int(d.get("seed", 1))
        arr[k].replicate_id = int(d.get("replicate_id", 0))
        arr[k].regime = int(d.get("regime", WF))
        arr[k].n0 = n0
        arr[k].capacity = int(d.get("capacity", n0))
        arr[k].n_loci = int(d.get("n_loci", 64))
        arr[k].n_patches = int(d.get("n_patches", 1))
        for f in ("mu", "r", "theta", "omega", "K", "fecundity", "migration", "home_return"):
            setattr(arr[k], f, float(d.get(f, 0.5 if f == "r" else 0.0)))
        arr[k].dispersal = int(d.get("dispersal", RING))
        arr[k].genetics = int(d.get("genetics", BIALLELIC))
        for f in ("allele_mean", "allele_sd", "mut_sd_factor", "noise_sd"):
            setattr(arr[k], f, float(d.get(f, 0.0)))
        arr[k].exp_transform = int(d.get("exp_transform", 0))
        for f in ("sexes", "mating", "monogamy"):
            setattr(arr[k], f, int(d.get(f, 0)))
        for f in ("pref_optimum", "pref_width"):
            setattr(arr[k], f, float(d.get(f, 0.0)))
        if d.get("physiology") is not None:
            ph = make_physiology(d["physiology"])
            keep.append(ph)
            arr[k].physiology = C.pointer(ph)
        if d.get("linkage") is not None:
            lk = np.ascontiguousarray(d["linkage"], dtype=np.float64)
            keep.append(lk)
            arr[k].linkage = _p(lk, C.c_double)
        eff = d.get("effects")
        if eff is not None:
            e = np.ascontiguousarray(eff, dtype=np.int8)
            keep.append(e)
            arr[k].effects = _p(e, C.c_int8)
        if d.get("ecology") is not None:
            eco = make_ecology(d["ecology"])
            keep.append(eco)
            arr[k].ecology = C.pointer(eco)
    return arr, keep


def footprint(reps):
    arr, _keep = make_descs(reps)
    n = load().spegg_footprint(arr, len(reps))
    if n == 0:
        raise SpeggError(E_INVALID, last_error())
    return int(n)


def threshold_table(kind, a, b=0, cap=None):
    cap = cap or max(1024, int(b) + 1)
    out = np.zeros(cap, dtype=np.uint64)
    n = load().spegg_threshold_table(int(kind), float(a), int(b), _p(out, C.c_uint64), cap)
    if n < 0:
        raise SpeggError(E_INVALID, "threshold_table rejected its arguments")
    return out[:n].copy()


def recomb_mode(r):
    return {0: "raw", 1: "zero", 2: "skip", 3: "lazy"}[load().spegg_recomb_mode(float(r))]


def geometric_gap(r, n_loci, x, guess):
    """(gap, table length) the offspring kernel's gap lookup gives for word
    x, searching from the first guess (host run of the same code)."""
    g = C.c_uint32(0)
    n = load().spegg_geometric_gap(float(r), int(n_loci), int(x), int(guess), C.byref(g))
    if n < 0:
        raise SpeggError(E_INVALID, "geometric_gap rejected its arguments")
    return int(g.value), int(n)


def philox_fill(seed, ctr):
    """Device Philox4x32-10 of counters ctr (n x 4 uint32) -> n x 4 uint32."""
    import torch
    c = torch.as_tensor(np.ascontiguousarray(ctr, dtype=np.uint32).view(np.int32)).reshape(-1, 4).to("cuda")
    out = torch.empty_like(c)
    stream = torch.cuda.current_stream().cuda_stream
    check(load().spegg_philox_fill(int(seed), c.data_ptr(), out.data_ptr(), c.shape[0], stream))
    return out.cpu().numpy().view(np.uint32)


def philox_rate(seed, blocks_per_thread, out):
    """Philox throughput probe on the current stream (no wait): out[i] =
    XOR of the words of blocks (i, k, 0, 0), k < blocks_per_thread; out is a
    device int32 tensor of n entries."""
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    check(load().spegg_philox_rate(int(seed), int(blocks_per_thread), out.data_ptr(), out.numel(), stream))


class Population:
    """Replicates resident in device memory, advanced by the HIP kernels.
    Per-patch accessors take ``patch`` (0 for single-patch replicates)."""

    def __init__(self, reps, device="cuda", stream=None):
        import torch
        self.lib = load()
        self.reps = [dict(d) for d in reps]
        self.n_reps = len(reps)
        arr, keep = make_descs(self.reps)
        self.footprint = int(self.lib.spegg_footprint(arr, self.n_reps))
        if self.footprint == 0:
            raise SpeggError(E_INVALID, last_error())
        self.workspace = torch.empty(self.footprint, dtype=torch.uint8, device=device)
        if stream is None:
            # a stream of its own (default priority), so generations can be
            # replayed as graphs; it waits for the workspace allocation
            stream = torch.cuda.Stream(device=self.workspace.device)
            stream.wait_stream(torch.cuda.current_stream(self.workspace.device))
        self.stream = stream
        h = C.c_void_p()
        check(self.lib.spegg_pop_create(arr, self.n_reps, C.c_void_p(self.workspace.data_ptr()), self.footprint,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.L = [int(d.get("n_loci", 64)) for d in self.reps]
        self.W = [(L + 31) // 32 for L in self.L]
        self.P = [int(d.get("n_patches", 1)) for d in self.reps]
        # demes per replicate: its patches, or the two species of the consumer-resource regime
        self.D = [2 if d.get("regime") == CONSUMER_RESOURCE else p for d, p in zip(self.reps, self.P)]
        self._owned = True
        del keep

    @classmethod
    def view(cls, handle, reps):
        """A non-owning view of a population handle held elsewhere (a kept
        job of the server); close() leaves the handle alone."""
        self = cls.__new__(cls)
        self.lib = load()
        self.reps = [dict(d) for d in reps]
        self.n_reps = len(reps)
        self.workspace, self.stream, self.footprint = None, None, None
        self._h = handle
        self._owned = False
        self.L = [int(d.get("n_loci", 64)) for d in self.reps]
        self.W = [(L + 31) // 32 for L in self.L]
        self.P = [int(d.get("n_patches", 1)) for d in self.reps]
        self.D = [2 if d.get("regime") == CONSUMER_RESOURCE else p for d, p in zip(self.reps, self.P)]
        return self

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owned", True):
                self.lib.spegg_pop_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, n=1):
        check(self.lib.spegg_step_generations(self._h, int(n)))

    def stats(self):
        out = (RepStats * self.n_reps)()
        check(self.lib.spegg_stats(self._h, out, self.n_reps))
        return [s.as_dict() for s in out]

    def deme_stats(self, rep=0):
        """The census of each of replicate rep's demes (patches, or species
        0 resource and 1 consumer)."""
        out = (RepStats * self.D[rep])()
        check(self.lib.spegg_deme_stats(self._h, rep, out, self.D[rep]))
        return [s.as_dict() for s in out]

    def _n_of(self, rep, patch=0, species=0):
        per = self.deme_stats(rep)
        k = patch + species
        if not 0 <= k < len(per):
            raise SpeggError(E_INVALID, f"deme {k} out of range (replicate {rep} has {len(per)})")
        return per[k]["n"]

    def genomes(self, rep=0, patch=0, species=0):
        n = self._n_of(rep, patch, species)
        W = self.W[rep]
        out = np.zeros(max(n, 1) * 2 * W, dtype=np.uint32)
        got = C.c_uint32()
        check(self.lib.spegg_read_genomes(self._h, rep, patch, species, _p(out, C.c_uint32), out.size,
                                          C.byref(got)))
        return out[: got.value * 2 * W].reshape(got.value, 2, W)

    def write_genomes(self, rep, words, generation, patch=0, species=0):
        w = np.ascontiguousarray(words, dtype=np.uint32).reshape(-1)
        n = w.size // (2 * self.W[rep])
        check(self.lib.spegg_write_genomes(self._h, rep, patch, species, _p(w, C.c_uint32), n, int(generation)))

    def phenotypes(self, rep=0, patch=0, species=0):
        n = self._n_of(rep, patch, species)
        out = np.zeros(max(n, 1), dtype=np.int32)
        got = C.c_uint32()
        check(self.lib.spegg_read_phenotypes(self._h, rep, patch, species, _p(out, C.c_int32), out.size,
                                             C.byref(got)))
        return out[: got.value]

    def alleles(self, rep=0, patch=0):
        """Continuous allelic values of a patch, shape (n, 2, L) float32."""
        n = self._n_of(rep, patch)
        L = self.L[rep]
        out = np.zeros(max(n, 1) * 2 * L, dtype=np.float32)
        got = C.c_uint32()
        check(self.lib.spegg_read_alleles(self._h, rep, patch, _p(out, C.c_float), out.size, C.byref(got)))
        return out[: got.value * 2 * L].reshape(got.value, 2, L)

    def write_alleles(self, rep, values, generation, patch=0):
        v = np.ascontiguousarray(values, dtype=np.float32).reshape(-1)
        n = v.size // (2 * self.L[rep])
        check(self.lib.spegg_write_alleles(self._h, rep, patch, _p(v, C.c_float), n, int(generation)))

    def phenotypes_f(self, rep=0, patch=0):
        """Continuous alleles: expressed phenotypes, float32."""
        n = self._n_of(rep, patch)
        out = np.zeros(max(n, 1), dtype=np.float32)
        got = C.c_uint32()
        check(self.lib.spegg_read_phenotypes_f(self._h, rep, patch, _p(out, C.c_float), out.size, C.byref(got)))
        return out[: got.value]

    def body(self, rep=0):
        """Physiology regime: (X, Y) float64, irreversible and reversible mass."""
        n = self._n_of(rep)
        X = np.zeros(max(n, 1), dtype=np.float64)
        Y = np.zeros(max(n, 1), dtype=np.float64)
        got = C.c_uint32()
        check(self.lib.spegg_read_body(self._h, rep, _p(X, C.c_double), _p(Y, C.c_double), X.size, C.byref(got)))
        return X[: got.value], Y[: got.value]

    def sexes(self, rep=0, patch=0):
        """Separate sexes: 0 female, 1 male, per individual (all 0 without sexes)."""
        n = self._n_of(rep, patch)
        out = np.zeros(max(n, 1), dtype=np.uint8)
        got = C.c_uint32()
        check(self.lib.spegg_read_sexes(self._h, rep, patch, _p(out, C.c_uint8), out.size, C.byref(got)))
        return out[: got.value]

    def ages(self, rep=0, species=0):
        n = self._n_of(rep, 0, species)
        out = np.zeros(max(n, 1), dtype=np.uint8)
        got = C.c_uint32()
        check(self.lib.spegg_read_ages(self._h, rep, species, _p(out, C.c_uint8), out.size, C.byref(got)))
        return out[: got.value]

    def intake(self, rep=0):
        """Consumers' credited captures in the last generation, by adult index."""
        n = self.deme_stats(rep)[1]["n_parents"]
        out = np.zeros(max(n, 1), dtype=np.uint32)
        got = C.c_uint32()
        check(self.lib.spegg_read_intake(self._h, rep, _p(out, C.c_uint32), out.size, C.byref(got)))
        return out[: got.value]

    def survivors(self, rep=0, patch=0, species=0):
        n = self.deme_stats(rep)[patch + species]["n_survivors"]
        out = np.zeros(max(n, 1), dtype=np.uint32)
        got = C.c_uint32()
        check(self.lib.spegg_read_survivors(self._h, rep, patch, species, _p(out, C.c_uint32), out.size,
                                            C.byref(got)))
        return out[: got.value]

    def allele_counts(self, rep=0, patch=0, species=0):
        """Copies of allele 1 per locus over a deme's current census (uint32, L)."""
        import torch
        L = self.L[rep]
        scratch = torch.empty(L, dtype=torch.int32, device=self.workspace.device)
        out = np.zeros(L, dtype=np.uint32)
        got = C.c_uint32()
        check(self.lib.spegg_allele_counts(self._h, rep, patch, species, C.c_void_p(scratch.data_ptr()),
                                           _p(out, C.c_uint32), L, C.byref(got)))
        return out

    def allele_counts_noalloc(self, rep=0, patch=0, species=0):
        """As allele_counts, with the library's own device counters (the
        call allocates no device memory)."""
        L = self.L[rep]
        out = np.zeros(L, dtype=np.uint32)
        got = C.c_uint32()
        check(self.lib.spegg_allele_counts_noalloc(self._h, rep, patch, species, _p(out, C.c_uint32), L,
                                                   C.byref(got)))
        return out

    def autotune(self, generations_per_trial=2):
        """Time the offspring kernel's shapes on real generations and keep the
        fastest per genome length; returns {W: lanes-per-gamete cap}.  The
        population advances by the trial generations (4 x
        generations_per_trial per shape and genome length)."""
        cap = 16
        w = np.zeros(cap, np.uint32)
        g = np.zeros(cap, np.uint32)
        n = C.c_uint32()
        check(self.lib.spegg_autotune(self._h, int(generations_per_trial), _p(w, C.c_uint32), _p(g, C.c_uint32), cap,
                                      C.byref(n)))
        return {int(w[k]): int(g[k]) for k in range(min(n.value, cap))}

    def set_offspring_cap(self, W, gcap):
        """Pin the offspring kernel's cap on lanes per gamete for genome
        length W words (what autotune would pick), without timing."""
        check(self.lib.spegg_set_offspring_cap(self._h, int(W), int(gcap)))

    def set_graph(self, enable=True):
        """Replay generations as captured HIP graphs (default) or launch eagerly."""
        check(self.lib.spegg_set_graph(self._h, 1 if enable else 0))

    def set_trace(self, enable=True):
        check(self.lib.spegg_set_trace(self._h, 1 if enable else 0))

    def parents(self, rep=0, patch=0, with_source=False, species=0):
        """Mother and father of each newborn of the last generation (indices
        into the adults of the patch it came from) and, with_source, that
        patch."""
        n = self._n_of(rep, patch, species)
        mom = np.zeros(max(n, 1), dtype=np.uint32)
        dad = np.zeros(max(n, 1), dtype=np.uint32)
        src = np.zeros(max(n, 1), dtype=np.uint32)
        got = C.c_uint32()
        check(self.lib.spegg_read_parents(self._h, rep, patch, species, _p(mom, C.c_uint32), _p(dad, C.c_uint32),
                                          _p(src, C.c_uint32), mom.size, C.byref(got)))
        if with_source:
            return mom[: got.value], dad[: got.value], src[: got.value]
        return mom[: got.value], dad[: got.value]

    def set_timing(self, kernels=("survive", "compact", "offspring", "encounter", "carry")):
        """Bracket the named kernels with HIP events (empty: stop)."""
        mask = 0
        for k in kernels:
            mask |= 1 << KERNEL_NAMES.index(k)
        check(self.lib.spegg_set_timing(self._h, mask))

    def prepare_graphs(self):
        """Capture and upload the generation graphs before they are replayed."""
        check(self.lib.spegg_prepare_graphs(self._h))

    def offspring_class_times(self):
        """[(W min, W max, ms summed, launches)] per offspring launch class
        since the last call."""
        cap = 64
        lo, hi = (C.c_uint32 * cap)(), (C.c_uint32 * cap)()
        ms, n = (C.c_double * cap)(), (C.c_uint64 * cap)()
        k = C.c_uint32()
        check(self.lib.spegg_offspring_class_times(self._h, lo, hi, ms, n, cap, C.byref(k)))
        return [(lo[i], hi[i], ms[i], n[i]) for i in range(min(k.value, cap))]

    def kernel_times(self):
        """{kernel: (ms summed, launches)} since the last call."""
        k = len(KERNEL_NAMES)
        ms = (C.c_double * k)()
        n = (C.c_uint64 * k)()
        check(self.lib.spegg_kernel_times(self._h, ms, n, k))
        return {KERNEL_NAMES[i]: (ms[i], n[i]) for i in range(k)}


class Server:
    """Sweep jobs served from one device arena with continuous batching
    (the library's native scheduler; this class only marshals arguments).

    ``arena`` is a device pointer (int) and its size, or None to allocate
    ``arena_bytes`` with torch.  Without a device (``arena`` given as a
    plain aligned integer) only submission checks can run."""

    def __init__(self, arena_bytes, arena=None, stream=None, device="cuda", n_streams=4):
        self.lib = load()
        self.workspace = None
        if arena is None:
            import torch
            self.workspace = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
            arena = self.workspace.data_ptr()
            if stream is None:
                stream = torch.cuda.Stream(device=self.workspace.device)
                stream.wait_stream(torch.cuda.current_stream(self.workspace.device))
        self.stream = stream
        sptr = stream.cuda_stream if stream is not None and hasattr(stream, "cuda_stream") else stream
        h = C.c_void_p()
        check(self.lib.spegg_server_create(C.c_void_p(int(arena)), int(arena_bytes), C.c_void_p(sptr),
                                           int(n_streams), C.byref(h)))
        self._h = h
        self.n_reps = {}

    def close(self):
        if getattr(self, "_h", None):
            self.lib.spegg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, job_id, reps, generations):
        arr, keep = make_descs(reps)
        check(self.lib.spegg_server_submit(self._h, int(job_id), arr, len(reps), int(generations)))
        self.n_reps[int(job_id)] = len(reps)
        self.descs = getattr(self, "descs", {})
        self.descs[int(job_id)] = [dict(d) for d in reps]
        del keep

    def step(self, generations=1):
        """One scheduling step; returns (resident, waiting).  Jobs that
        finished in this step are retired (polled) at a later step or drain."""
        res, wait = C.c_uint32(), C.c_uint32()
        check(self.lib.spegg_server_step(self._h, int(generations), C.byref(res), C.byref(wait)))
        return res.value, wait.value

    def drain(self):
        """Wait for all enqueued work, retire finished jobs, then admit."""
        return self.step(0)

    def keep(self, job_id):
        """Hold the job's population after it finishes (until release)."""
        check(self.lib.spegg_server_keep(self._h, int(job_id)))

    def population(self, job_id):
        """A view of a finished, kept job's population (genomes etc.)."""
        h = C.c_void_p()
        check(self.lib.spegg_server_population(self._h, int(job_id), C.byref(h)))
        return Population.view(h, self.descs[int(job_id)])

    def release(self, job_id):
        check(self.lib.spegg_server_release(self._h, int(job_id)))

    def poll(self, cap=1024):
        ids = (C.c_uint64 * cap)()
        n = C.c_uint32()
        check(self.lib.spegg_server_poll(self._h, ids, cap, C.byref(n)))
        return [int(ids[i]) for i in range(n.value)]

    def result(self, job_id):
        n = self.n_reps[int(job_id)]
        out = (RepStats * n)()
        check(self.lib.spegg_server_result(self._h, int(job_id), out, n))
        del self.n_reps[int(job_id)]
        return [x.as_dict() for x in out]

    def usage(self):
        used, free = C.c_size_t(), C.c_size_t()
        check(self.lib.spegg_server_usage(self._h, C.byref(used), C.byref(free)))
        return used.value, free.value
