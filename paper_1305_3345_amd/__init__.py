"""MI355X-native batched AES (CBC, CTR) over page-sized buffers.

The compute path is libaesgpu.so (HIP kernels for gfx950 behind a C ABI, see
include/aesgpu.h); ``aesgpu`` is its ctypes binding.
"""
from . import aesgpu  # noqa: F401
from .aesgpu import (AES_DEVICE_NONE, AES_OP_CBC_DEC, AES_OP_CBC_ENC, AES_OP_CTR,  # noqa: F401
                     AesError, Context, Graph, Plan, batch, cbc_decrypt_batch, cbc_encrypt_batch,
                     ctr_batch, expand_key, expand_keys, request_launch, Server,
                     schedules_to_device, tune)
