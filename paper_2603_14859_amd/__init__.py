"""MI355X (gfx950) library for voxelwise ABC rejection in dynamic PET (vPET-ABC).

The work is done by hand-written HIP kernels in ``libvpetabc.so`` behind the C
ABI of ``include/vpet_abc.h``; this package is the thin ctypes binding with the
same entry points (``simulate``, ``infer``, ``infer_noalloc``, ``draws``, ``accept_count``, the
shared-bank ``bank_build`` / ``infer_bank`` / ``stream_bank``, the learned
proposal ``proposal_init`` / ``proposal_forward`` / ``proposal_loss_grad`` /
``proposal_train`` and the shared bank drawn from it, ``infer_bank_learned`` /
``stream_bank_learned``).
"""
from ._binding import (E_ARG, E_GRID, E_HIP, E_LIMIT, E_MODEL, E_NOMEM, EXPORTED, LIB_PATH, M_1TCM,  # noqa: F401
                       M_2TCM_IRR, M_2TCM_REV, M_LPNTPET, M_MRTM, MAX_ACCEPT, OK, PSTRIDE, VpetError, accept_count, draws, infer,
                       lib, model_mask, simulate, version, bank_build, infer_bank, BANK_MAX_ACCEPT, BANK_MAX_FRAMES,
                       stream_bank, load_stream_outputs, E_IO, PROPOSAL_NPARAM, PROPOSAL_NOUT,
                       PROPOSAL_MAX_FRAMES, proposal_init, proposal_forward, proposal_loss_grad, proposal_train,
                       infer_noalloc, bank_screen, infer_bank_learned,
                       stream_bank_learned)
