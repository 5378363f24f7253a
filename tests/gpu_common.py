"""Shared helpers of the GPU parity tests (library through the C-ABI vs oracle)."""
import numpy as np

from oracle import ref
from paper_2508_12093_amd import ffi


class Pair:
    """A library context and an oracle for the same preset and seeds."""

    def __init__(self, name, key_seed=11, relin_seed=12, galois_seed=13, steps=(1, 3, 5)):
        self.name = name
        self.ctx = ffi.ppst_context_create(name)
        self.P = ref.Params.preset(name)
        self.O = ref.Oracle(self.P)
        self.info = self.ctx.info
        self.sk, self.pk = ffi.ppst_keygen(self.ctx, key_seed)
        self.osk, self.opk = self.O.keygen(key_seed)
        self.evk = ffi.ppst_evk_create(self.ctx)
        ffi.ppst_evk_add_relin(self.ctx, self.sk, relin_seed, self.evk)
        self.orlk = self.O.relin_key(self.osk, relin_seed)
        self.steps = list(steps)
        ffi.ppst_evk_add_galois(self.ctx, self.sk, self.steps, galois_seed, self.evk)
        self.ogk = self.O.rotation_keys(self.osk, galois_seed, self.steps)
        self.galois_seed = galois_seed

    def add_rotsum_keys(self):
        if getattr(self, "_rotsum_keys", False):
            return
        self._rotsum_keys = True
        ffi.ppst_evk_add_rotsum(self.ctx, self.sk, self.galois_seed, self.evk)
        need = [r for r in self.O.rotsum_hoisted8_steps() if ref.galois_element(r, self.P.N) not in self.ogk]
        self.ogk.update(self.O.rotation_keys(self.osk, self.galois_seed, need))

    def encrypt(self, values, seed, level=None):
        level = self.P.L if level is None else level
        pt = ffi.ppst_encode(self.ctx, values, level)
        ct = ffi.ppst_encrypt(self.ctx, self.pk, pt, seed)
        oct_ = self.O.encrypt(self.O.encode(values, level), self.opk, seed)
        return ct, oct_

    def export(self, ct):
        return ffi.ppst_ct_export(self.ctx, ct)

    def same(self, ct, oct_):
        got = self.export(ct)
        assert ct.level == oct_.level, (ct.level, oct_.level)
        assert ct.scale == oct_.scale
        assert got.shape == oct_.data.shape, (got.shape, oct_.data.shape)
        diff = int(np.sum(got != oct_.data))
        assert diff == 0, "%d of %d residues differ" % (diff, got.size)

    def decrypt(self, ct, n=None):
        pt = ffi.ppst_decrypt(self.ctx, self.sk, ct)
        return ffi.ppst_decode(self.ctx, pt, n)
