// Host-side helper shared by the readout library: pack FP32 network parameters
// [n_obj][15681] into the per-object BF16 MFMA images (layout in nsdf_device.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

hipError_t nsdf_pack_images(const float* params, int n_obj, uint32_t* images, hipStream_t stream);
