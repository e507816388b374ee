// fvv_unet.h -- the learned blend/inpaint network of libfvv.so: a 4-level
// U-Net (widths 32/64/128/256) over the 16-channel warped-camera stack,
// bf16 activations and weights on the matrix cores with fp32 accumulation,
// fp32 master weights and Adam for training.  Internal to the library.
//
// A network (weights, Adam moments, gradient) is shared by every stream of a
// context; each stream that runs it owns an activation set.  All calls
// enqueue on the given stream; functions that return host data synchronise it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#define UNET_IN 16          // stack channels on the device (15 used, one zero channel)
#define UNET_ALIGN 8        // network inputs are padded to multiples of 8 in both dimensions

struct unet_layer {
    const char *name;
    int kind;                  // 0 conv3x3 + ReLU, 1 convT 2x2, 2 head 1x1
    int cin, cout;             // canonical channels
    int cin_pad;               // device input channels (multiple of 32, except the head)
    int taps;                  // 9, 4 or 1
    size_t w_off, b_off;       // float offsets into the parameter vector
    size_t wf_off, wd_off;     // bf16 offsets of the forward / data-gradient layouts
};

struct unet_state;
struct unet_act;

unet_state *unet_new();
void unet_free(unet_state *n);
unet_act *unet_act_new();
void unet_act_free(unet_act *a);
size_t unet_param_floats();
int unet_layer_count();
const unet_layer *unet_layer_info(int i);
size_t unet_weight_bytes();                            // device bytes of a loaded network
size_t unet_act_need(size_t pixels, bool train);       // device bytes of an activation set
size_t unet_act_bytes(const unet_act *a);              // bytes it holds now
size_t unet_act_cap(const unet_act *a);                // pixels it holds now
bool unet_act_trainable(const unet_act *a);            // holds the training buffers
bool unet_loaded(const unet_state *n);

// Upload canonical fp32 parameters (layer order, weights (C_out, kh, kw,
// C_in) then bias), reset Adam, prepare the bf16 copies.
hipError_t unet_set_params(unet_state *n, const float *host, hipStream_t s);
hipError_t unet_get_params(unet_state *n, float *host, hipStream_t s);
hipError_t unet_get_grads(unet_state *n, float *host, hipStream_t s);
// Make the activation set hold B*H*W pixels (grows only; synchronises the
// device when it reallocates).
hipError_t unet_act_reserve(unet_act *a, size_t pixels, bool train);
// Forward over a stack [B][H][W][16] bf16 (H, W multiples of 8).  Writes
// s = sigmoid output fp32 [B][H][W][3] to s_out if non-null and, if rgb is
// non-null, RGB8 of the first valid_h rows and valid_w columns of image b at
// rgb + b * img_stride (pitch bytes per row), for every pixel whose three
// outputs are finite (the others keep what the buffer held).
// keep: store every layer's output (for unet_read_act); otherwise the
// finest transposed convolution may run inside the convolution after it,
// and the head inside the last convolution, neither of their inputs stored.
hipError_t unet_forward(unet_state *n, unet_act *a, const uint16_t *stack, int B, int H, int W, float *s_out,
                           uint8_t *rgb, int64_t pitch, int64_t img_stride, int valid_h, int valid_w,
                           hipStream_t s, std::string &err, bool keep = true);
// RGB8 destination of image b of a batched forward: its first h rows and w
// columns at rgb, pitch bytes per row (32 bytes, so a table of them copies
// in 16-byte words).
struct unet_out {
    uint8_t *rgb;
    int64_t pitch;
    int32_t h, w;
    int64_t pad;
};
// Forward over B stacks of one size with per-image RGB8 destinations
// (outs: B entries in device memory); pixels whose three outputs are not
// finite keep what the destination held.  Each image's result is the same
// for any B (the per-output accumulation order does not depend on the batch).
hipError_t unet_forward_batch(unet_state *n, unet_act *a, const uint16_t *stack, int B, int H, int W,
                              const unet_out *outs, hipStream_t s, std::string &err, bool keep = true);
// One training step: forward, L1 loss against target fp32 [B][H][W][3] over
// rows < valid_h, backward into the gradient; apply != 0 then takes one Adam
// step with learning rate lr (apply == 0 leaves the parameters unchanged).
// The mean loss is written to *loss_host if non-null.
hipError_t unet_train(unet_state *n, unet_act *a, const uint16_t *stack, const float *target, int B, int H,
                         int W, int valid_h, float lr, int apply, float *loss_host, hipStream_t s,
                         std::string &err);
// Copy one layer's stored output of the last forward (bf16 NHWC, that
// layer's channels only) to host memory, for parity checks; an error for
// a layer (the finest transposed convolution, dec0b) whose output the last
// forward did not store.
hipError_t unet_read_act(unet_act *a, int layer, void *host, size_t bytes, hipStream_t s);
// Adds to *bad_dev (device memory) the number of non-NaN float32 bit
// patterns whose bfloat16 rounding by the hardware conversion the kernels
// use differs from round-to-nearest-even written out on the bits.
hipError_t unet_check_bf16(unsigned long long *bad_dev, hipStream_t s);
