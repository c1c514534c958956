"""Oracle streams with a planted start block, mirroring the library's test hook
SFD_OPT_TEST_ZERO_ROW: row j of the start block G of SimultaneousIteration (Alg 1) is set to 0
in the attempts a < zero_attempts of every buffer step, so a buffer whose dominant direction is
e_j gets a SparseShrink that VerifySpectral (Alg 6) rejects and BoostedSparseShrink (Alg 4)
retries."""

from oracle import SFDOracle


class ZeroRowOracle(SFDOracle):
    def __init__(self, *args, zero_row=0, zero_attempts=1, **kw):
        super().__init__(*args, **kw)
        self.zero_row = int(zero_row)
        self.zero_attempts = int(zero_attempts)

    def draw_start_block(self, buffer_idx, attempt, purpose):
        G = super().draw_start_block(buffer_idx, attempt, purpose)
        if attempt < self.zero_attempts:
            G[self.zero_row, :] = 0.0
        return G
